// Device-side photon history: Philox stream, physics steps and the per-lane
// state machine shared by the transport, replay and adjoint kernels.
#pragma once

#include "mc_internal.h"

namespace mcs {
namespace {

constexpr uint32_t KAHN_MAX = 64;
constexpr float INV_MEC2 = (float)(1.0 / 510.99895);
constexpr double MEC2_D = 510.99895;

enum : int { S_IDLE = 0, S_EMIT0 = 1, S_EMIT1 = 2, S_STEP = 3, S_KAHN = 4 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// (words 0 and 2), xor-mixed with words 1 and 3 and the key; the key takes a
// Weyl step after every round.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
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

// Problem constants a wavefront works with (wave-uniform).
struct Cst {
    const float* mu;
    const uint32_t* q32;
    const uint64_t* cdf;
    const uint32_t* guide;
    const float2* views;
    int nx, ny, nz, source_mode;
    float hx, hy, hz, lx, ly, lz, inv_vox, vox;
    int nu, nv;
    float inv_pix, radius, cos_alpha, wu, wv, e_lo, e_hi, e_cut;
    float f_pe, mu_hat, inv_mm140, p_pe140;
    double kn140;
    uint32_t seed, pid, max_steps, shift;
    uint64_t total, q_per_view, r_extra, work_begin, tally_offset;
    uint32_t flags;
};

__device__ inline Cst load_cst(const ProbDesc* __restrict__ d) {
    Cst c;
    c.mu = d->mu;
    c.q32 = d->q32; c.cdf = d->cdf; c.guide = d->guide; c.views = d->views;
    c.nx = d->nx; c.ny = d->ny; c.nz = d->nz; c.source_mode = d->source_mode;
    c.hx = d->hx; c.hy = d->hy; c.hz = d->hz;
    c.lx = d->lx; c.ly = d->ly; c.lz = d->lz;
    c.inv_vox = d->inv_vox; c.vox = d->vox;
    c.nu = d->nu; c.nv = d->nv;
    c.inv_pix = d->inv_pix; c.radius = d->radius; c.cos_alpha = d->cos_alpha;
    c.wu = d->wu; c.wv = d->wv; c.e_lo = d->e_lo; c.e_hi = d->e_hi; c.e_cut = d->e_cut;
    c.f_pe = d->f_pe;
    c.mu_hat = __uint_as_float(d->mu_hat_bits);
    c.kn140 = d->kn140;
    // g(140 keV) = 1 by construction: mu_max(140) = max mu, p_pe(140) = f.
    c.inv_mm140 = (float)(1.0 / (double)c.mu_hat);
    c.p_pe140 = c.f_pe;
    c.seed = d->seed; c.pid = d->problem_id; c.max_steps = d->max_steps; c.shift = d->shift;
    c.total = d->total; c.q_per_view = d->q_per_view; c.r_extra = d->r_extra;
    c.work_begin = d->work_begin; c.tally_offset = d->tally_offset;
    c.flags = d->flags;
    return c;
}

// Attenuation scale g(E) and photoelectric probability at energy e, in double
// precision (once per scatter): g(E) = (1-f) KN(E)/KN(140) + f (140/E)^3.
__device__ inline double energy_terms(const Cst& C, float e, float& inv_mm, float& p_pe) {
    const double E = (double)e;
    const double k = E / MEC2_D;
    const double a = 1.0 + 2.0 * k;
    const double la = log(a);
    const double kn = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - la / k) + la / (2.0 * k)
                      - (1.0 + 3.0 * k) / (a * a);
    const double r = 140.0 / E;
    const double pe = (double)C.f_pe * r * r * r;
    const double g = (1.0 - (double)C.f_pe) * kn / C.kn140 + pe;
    inv_mm = (float)(1.0 / ((double)C.mu_hat * g));
    p_pe = (float)(pe / g);
    return g;
}

struct Lane {
    uint64_t hist, work;
    int view, state;
    uint32_t n, a, phi_word, emit_voxel;
    int n_scatter;
    float x, y, z, dx, dy, dz, e, inv_mm, p_pe, vc, vs;
};

// Per-lane accumulators of one problem (reduced across the wave on flush).
struct Acc {
    uint32_t fate[7];
    uint32_t n_tent, n_real, n_kahn, n_hist;
    long long e_dep, e_esc, e_cap;
};

__device__ inline void acc_zero(Acc& A) {
#pragma unroll
    for (int i = 0; i < 7; ++i) A.fate[i] = 0;
    A.n_tent = A.n_real = A.n_kahn = A.n_hist = 0;
    A.e_dep = A.e_esc = A.e_cap = 0;
}

__device__ __forceinline__ long long to_q23(float kev) {
    return __float2ll_rn(kev * 8388608.0f);
}

// Outcome of one iteration.
enum : int { R_RUNNING = -1 };

// Per-lane escape: collimator, detector bin, window.  Returns the fate; sets iu, iv.
__device__ inline int escape(const Cst& C, const Lane& L, int& iu, int& iv) {
    const float dn = L.dx * L.vc + L.dy * L.vs;
    if (dn < C.cos_alpha) return MC_ESCAPED;
    const float tp = (C.radius - (L.x * L.vc + L.y * L.vs)) / dn;
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

__device__ inline void rotate(Lane& L, float ct, float phi_u) {
    float sp, cp;
    sincospif(2.0f * phi_u, &sp, &cp);
    const float st = sqrtf(fmaxf(0.0f, (1.0f - ct) * (1.0f + ct)));
    const float u = L.dx, v = L.dy, w = L.dz;
    if (fabsf(w) > 0.99999f) {
        L.dx = st * cp;
        L.dy = st * sp;
        L.dz = w > 0.0f ? ct : -ct;
    } else {
        const float t = sqrtf((1.0f - w) * (1.0f + w));
        const float it = 1.0f / t;
        L.dx = st * (u * w * cp - v * sp) * it + u * ct;
        L.dy = st * (v * w * cp + u * sp) * it + v * ct;
        L.dz = -st * cp * t + w * ct;
    }
}

__device__ __forceinline__ void counter_of(const Lane& L, uint32_t& c2, uint32_t& c3) {
    c2 = 0; c3 = 0;
    if (L.state == S_EMIT1) c3 = 1;
    else if (L.state == S_STEP) c2 = L.n + 1;
    else if (L.state == S_KAHN) { c2 = L.n; c3 = 1 + L.a; }
}

// Start a history from its problem-local work index g.
__device__ inline void begin_history(const Cst& C, Lane& L, uint64_t g, uint64_t work) {
    const uint64_t big = C.q_per_view + 1;
    uint64_t view, hist;
    if (g < C.r_extra * big) { view = g / big; hist = g - view * big; }
    else {
        const uint64_t g2 = g - C.r_extra * big;
        view = C.r_extra + g2 / C.q_per_view;
        hist = g2 - (view - C.r_extra) * C.q_per_view;
    }
    L.hist = hist;
    L.view = (int)view;
    L.work = work;
    L.state = S_EMIT0;
    L.n = 0; L.a = 0; L.n_scatter = 0;
    const float2 cs = C.views[view];
    L.vc = cs.x; L.vs = cs.y;
}

// One iteration of a lane's history given its Philox words.  Returns the fate
// when the history ends (iu/iv set for escapes), else R_RUNNING.
__device__ inline int advance(const Cst& C, Lane& L, uint32_t w0, uint32_t w1, uint32_t w2,
                              uint32_t w3, Acc& A, int& iu, int& iv) {
    if (L.state == S_STEP) {
        L.n += 1;
        if (L.n > C.max_steps) {
            L.n -= 1;
            A.e_cap += to_q23(L.e);
            return MC_CAPPED_FATE;
        }
        A.n_tent++;
        const float s = -__logf(unif(w0)) * L.inv_mm;
        const float xn = fmaf(s, L.dx, L.x);
        const float yn = fmaf(s, L.dy, L.y);
        const float zn = fmaf(s, L.dz, L.z);
        const float tx = xn + C.hx, ty = yn + C.hy, tz = zn + C.hz;
        const bool inside = (tx >= 0.0f) & (tx < C.lx) & (ty >= 0.0f) & (ty < C.ly) &
                            (tz >= 0.0f) & (tz < C.lz);
        if (!inside) {
            A.e_esc += to_q23(L.e);
            return escape(C, L, iu, iv);
        }
        const int ix = min((int)(tx * C.inv_vox), C.nx - 1);
        const int iy = min((int)(ty * C.inv_vox), C.ny - 1);
        const int iz = min((int)(tz * C.inv_vox), C.nz - 1);
        const uint32_t q = C.q32[(uint32_t)ix + (uint32_t)C.nx * ((uint32_t)iy + (uint32_t)C.ny * (uint32_t)iz)];
        L.x = xn; L.y = yn; L.z = zn;
        if ((w1 >> 8) < q) {
            A.n_real++;
            if (unif(w2) < L.p_pe) {
                A.e_dep += to_q23(L.e);
                return MC_ABSORBED;
            }
            L.phi_word = w3;
            L.a = 0;
            L.state = S_KAHN;
        }
        return R_RUNNING;
    }
    if (L.state == S_KAHN) {
        A.n_kahn++;
        const float k = L.e * INV_MEC2;
        const float tk = 2.0f * k;
        const float r1 = unif(w0), r2 = unif(w1), r3 = unif(w2);
        float xx;
        bool acc;
        if (r1 <= (1.0f + tk) / (9.0f + tk)) {
            xx = fmaf(tk, r2, 1.0f);
            const float ix = 1.0f / xx;
            acc = r3 <= 4.0f * (ix - ix * ix);
        } else {
            xx = (1.0f + tk) / fmaf(tk, r2, 1.0f);
            const float c = 1.0f - (xx - 1.0f) / k;
            acc = r3 <= 0.5f * (c * c + 1.0f / xx);
        }
        if (!acc) {
            L.a += 1;
            if (L.a >= KAHN_MAX) {
                A.e_cap += to_q23(L.e);
                return MC_CAPPED_FATE;
            }
            return R_RUNNING;
        }
        const float ct = 1.0f - (xx - 1.0f) / k;
        const float en = L.e / xx;
        A.e_dep += to_q23(L.e - en);
        L.e = en;
        L.n_scatter += 1;
        rotate(L, ct, unif(L.phi_word));
        if (L.e < C.e_cut) {
            A.e_dep += to_q23(L.e);
            return MC_CUT;
        }
        energy_terms(C, L.e, L.inv_mm, L.p_pe);
        L.state = S_STEP;
        return R_RUNNING;
    }
    if (L.state == S_EMIT0) {
        // voxel by inverse CDF: t = floor(R * total / 2^64) with R the 64-bit word pair
        const uint64_t R = ((uint64_t)w0 << 32) | w1;
        const uint64_t t = __umul64hi(R, C.total);
        const uint64_t b = t >> C.shift;
        uint32_t lo = C.guide[b], hi = C.guide[b + 1];
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (C.cdf[mid] > t) hi = mid; else lo = mid + 1;
        }
        L.emit_voxel = lo;
        if (C.source_mode == MC_SOURCE_POINT) {
            L.x = 0.0f; L.y = 0.0f; L.z = 0.0f;
        } else {
            const uint32_t ix = lo % (uint32_t)C.nx;
            const uint32_t iy = (lo / (uint32_t)C.nx) % (uint32_t)C.ny;
            L.x = -C.hx + ((float)ix + unif(w2)) * C.vox;
            L.y = -C.hy + ((float)iy + unif(w3)) * C.vox;
        }
        L.state = S_EMIT1;
        return R_RUNNING;
    }
    // S_EMIT1: z position, direction, energy
    if (C.source_mode != MC_SOURCE_POINT) {
        const uint32_t iz = L.emit_voxel / ((uint32_t)C.nx * (uint32_t)C.ny);
        L.z = -C.hz + ((float)iz + unif(w0)) * C.vox;
    }
    const float ct = fmaf(2.0f, unif(w1), -1.0f);
    const float st = sqrtf((1.0f - ct) * (1.0f + ct));
    float sp, cp;
    sincospif(2.0f * unif(w2), &sp, &cp);
    L.dx = st * cp; L.dy = st * sp; L.dz = ct;
    L.e = 140.0f;
    L.inv_mm = C.inv_mm140;
    L.p_pe = C.p_pe140;
    L.n = 0;
    L.state = S_STEP;
    return R_RUNNING;
}

}  // namespace
}  // namespace mcs
