// Photon transport kernels for gfx950.
//
// One photon history per lane, followed from emission to absorption, energy
// cut or escape (history-by-history Monte Carlo, paper Sec. 2), then through
// an ideal parallel-hole collimator into a photopeak-window projection tally
// (Sec. 3).
//
// Execution model
//  * Every iteration of the main loop draws exactly one Philox4x32-10 block
//    per active lane.  The lane's state (tentative collision or Kahn attempt)
//    picks the counter and what the four words mean, so the dominant cost --
//    the 10 Philox rounds -- runs with all lanes in lockstep, and only the
//    short per-state tails diverge.
//  * Emission is converged: a wavefront emits the next 128 histories of its
//    chunk into an LDS stage in one phase (two per lane), and a lane whose
//    history ends starts the next staged one.  Chunks come from one global
//    atomic and never straddle problems, and a wavefront finishes the
//    histories of one problem before it starts another, so every problem
//    constant is wave-uniform (scalar registers) even in the batched launch.
//  * Fate counts, energies and work counters stay in registers and are
//    reduced across the wavefront before one atomic per value; tallies are
//    64-bit fixed-point integer atomics, so every sum is exact and
//    order-independent: results are bit-identical from run to run.
//  * Woodcock tracking: one threshold gather per tentative collision (a
//    one-byte palette code when the map allows, the palette in LDS); the
//    accept test is an integer compare.
//  * Forced detection (a second instantiation): the emission phase scores
//    each emitted history's forced copy; real collisions queue their forced
//    copies in a per-wave LDS ring that the wavefront scores 64 at a time, so
//    the long ray walks run converged rather than inside one lane's history.
#include "history.h"

namespace mcs {
namespace {

__device__ __forceinline__ uint32_t wsum32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
    return v;
}
// Lanes of mask m below this lane (two mbcnt instructions).
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Per-lane fate counts packed in 9-bit fields (fate f at bit 9 f), added to
// the wave-uniform counts fc and cleared: a lane ends at most one history
// per iteration, so a fold at least every 511 iterations keeps each field
// from overflowing.  All 64 lanes call.
constexpr uint32_t FATE_FOLD = 511;
__device__ inline void fold_fates(uint64_t& fpk, uint32_t* fc) {
#pragma unroll
    for (int f = 0; f < 7; ++f)
        fc[f] += __builtin_amdgcn_readfirstlane(wsum32((uint32_t)(fpk >> (9 * f)) & 511u));
    fpk = 0;
}

__device__ __forceinline__ long long wsum64(long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Wave-wide flush of one problem's accumulators (all 64 lanes must call).
// fc: wave-uniform fate counts; A: the lane's tentative collisions, real
// collisions and Kahn attempts (advance() counts them; summed here, which
// costs less than three ballots per iteration); e_esc: the lane's escaped
// energy (Q40.23);
// rays / pieces: the lane's forced-copy ray walks and the voxels they
// visited.  The deposited energy is filled in after the kernel (k_finalize).
// count_tallied: add the tallied histories to T.n_events (an analog run
// without an event list, whose count needs no per-history atomic).
__device__ inline void flush(long long& e_esc, uint32_t* fc, Acc& A, uint32_t& rays,
                             uint32_t& pieces, int p, const TransportArgs& T, int lane,
                             bool count_tallied) {
    const long long ee = wsum64(e_esc);
    const long long n_rays = wsum64(rays), n_pieces = wsum64(pieces);
    const long long n_tent = wsum64(A.n_tent), n_real = wsum64(A.n_real), n_kahn = wsum64(A.n_kahn);
    uint32_t nh = 0;
#pragma unroll
    for (int i = 0; i < 7; ++i) nh += fc[i];
    if (lane == 0 && nh > 0) {
        unsigned long long* fa = (unsigned long long*)(T.fates + (size_t)p * MC_N_FATES);
#pragma unroll
        for (int i = 0; i < 7; ++i) if (fc[i]) atomicAdd(fa + i, (unsigned long long)fc[i]);
        if (T.energy) atomicAdd((unsigned long long*)(T.energy + (size_t)p * 4 + 1), (unsigned long long)ee);
        if (count_tallied && fc[MC_TALLIED]) atomicAdd(T.n_events, (unsigned long long)fc[MC_TALLIED]);
        if (T.counters) {
            unsigned long long* ca = (unsigned long long*)(T.counters + (size_t)p * MC_N_COUNTERS);
            atomicAdd(ca + 0, (unsigned long long)n_tent);
            atomicAdd(ca + 1, (unsigned long long)n_real);
            atomicAdd(ca + 2, (unsigned long long)n_kahn);
            atomicAdd(ca + 3, (unsigned long long)nh);
            if (n_rays) {
                atomicAdd(ca + 4, (unsigned long long)n_rays);
                atomicAdd(ca + 5, (unsigned long long)n_pieces);
            }
        }
        if (fc[MC_CAPPED_FATE]) {
            atomicOr((unsigned long long*)T.status, (unsigned long long)MC_STATUS_CAPPED);
            atomicAdd((unsigned long long*)(T.status + 1), (unsigned long long)fc[MC_CAPPED_FATE]);
        }
    }
    e_esc = 0;
    rays = pieces = 0;
#pragma unroll
    for (int i = 0; i < 7; ++i) fc[i] = 0;
    acc_zero(A);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ long long readlane64(long long v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)(unsigned long long)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((unsigned long long)v >> 32), l);
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Wavefront-aggregated fixed-point tally: the lanes of mask m (wave-uniform)
// add w (and w2 into the squared tally) to bin off + bin; lanes with equal
// bins are summed first (one 64-bit atomic per distinct bin and array).
// Integer sums: the result is the same as one atomic per lane.  All lanes
// call; the loop runs once per distinct bin.
__device__ inline void tally_aggregated(const TransportArgs& T, size_t off, uint64_t m, uint32_t bin,
                                        long long w, long long w2, int lane) {
    while (m != 0) {
        const int lead = __builtin_ctzll(m);
        const uint32_t key = __builtin_amdgcn_readlane(bin, lead);
        const uint64_t grp = __ballot(bin == key) & m;
        long long s = 0, s2 = 0;
        for (uint64_t g = grp; g != 0; g &= g - 1) {
            const int l = __builtin_ctzll(g);
            s += readlane64(w, l);
            s2 += readlane64(w2, l);
        }
        if (lane == lead) {
            atomicAdd((unsigned long long*)(T.tally + off + key), (unsigned long long)s);
            if (T.tally_sq) atomicAdd((unsigned long long*)(T.tally_sq + off + key), (unsigned long long)s2);
        }
        m &= ~grp;
    }
}

// Problem-local work index of (view, hist): view-major order.
__device__ __forceinline__ uint64_t work_of(const Cst& C, uint64_t view, uint64_t hist) {
    return view * C.q_per_view + min(view, C.r_extra) + hist;
}

// Emission records a wavefront stages in LDS: four per lane (one in the
// forced-detection modes, whose LDS also holds the copy and job queues).
// Fewer, longer emission phases: two per lane measured 1.6 % slower on the
// headline thorax, five the same as four.
constexpr int EMIT_PER_LANE = 4;
constexpr int EMIT_BATCH = 64 * EMIT_PER_LANE;
constexpr int emit_per_lane(int mode) { return mode == 1 || mode == 2 ? 1 : EMIT_PER_LANE; }
constexpr int WAVES_PER_BLOCK_MAX = 4;    // 256 threads

struct EmitRec {
    float x, y, z, dx, dy, dz;
    uint32_t voxel, view, hist;
    float vc, vs;       // the view's detector normal, read in the converged emission phase
};

constexpr uint32_t FD_RING = 128;         // forced-detection queue per wave
constexpr uint32_t FD_JOBS = 128;         // scoring jobs waiting for their walks, per wave
// Events of listed forced copies staged per wave before one atomic appends
// them: the list's counter is one address for the whole device, so one
// atomic per few hundred events instead of one per scored batch.
constexpr uint32_t EV_STAGE = 160;

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Append the wave's staged events to the list: one atomic reserves `count`
// slots, the lanes copy the stage out; slots past the capacity are dropped
// but counted, as for a direct append.  All 64 lanes call; count is
// wave-uniform.
__device__ inline void flush_events(const TransportArgs& T, const mc_event* stage, uint32_t& count,
                                    int lane) {
    if (count == 0) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(T.n_events, (unsigned long long)count);
    base = uniform64(base);
    wave_sync_lds();
    for (uint32_t i = (uint32_t)lane; i < count; i += 64) {
        const uint64_t idx = base + i;
        if (idx < T.event_capacity) T.events[idx] = stage[i];
    }
    wave_sync_lds();
    count = 0;
}

// The set-up of one forced copy for this mode (false: it scores nothing).
template <int MODE>
__device__ __forceinline__ bool fd_setup_mode(const Cst& C, const ProbDesc* __restrict__ d, const FdPoint& q,
                                              FdJob& j) {
    if constexpr (MODE == 2) return cfd_setup(C, d, q, j);
    else return fd_setup(C, d, q, j);
}

// Walk and score the job of each lane with valid set: tally (Q31.32), sum of
// squares (Q11.52) and, if listed, one event each into the wave's stage
// (ev_count more; the caller keeps room for 64); convolution-based forced
// detection deposits into the depth layer instead (no events, no sum of
// squares).  All 64 lanes call.
template <int MODE>
__device__ inline void fd_score(const Cst& C, int p, const FdJob& j, bool valid, int lane,
                                const TransportArgs& T, uint32_t& rays, uint32_t& pieces,
                                mc_event* stage, uint32_t& ev_count) {
    uint32_t pc = 0;
    float sc = 0.0f;
    if (valid) sc = fd_walk_score(C, j, pc);
    rays += pc != 0;
    pieces += pc;
    if constexpr (MODE == 2) {
        if (valid) {
            const uint64_t lb = ((uint64_t)j.bin_hi << 32) | j.bin_lo;
            atomicAdd((unsigned long long*)(T.descs[p].layers + lb),
                      (unsigned long long)signed_weight(T.descs + p, j.voxel,
                                                        __float2ll_rn(sc * 4294967296.0f)));
        }
        return;
    }
    long long w = 0;
    if (valid) {
        w = signed_weight(T.descs + p, j.voxel, __float2ll_rn(sc * 4294967296.0f));
        const size_t b = C.tally_offset + j.bin_lo;
        atomicAdd((unsigned long long*)(T.tally + b), (unsigned long long)w);
        if (T.tally_sq)
            atomicAdd((unsigned long long*)(T.tally_sq + b),
                      (unsigned long long)__float2ll_rn(sc * sc * 4503599627370496.0f));
    }
    if (T.events) {            // forced copies are counted only when listed
        const uint64_t m = __ballot(valid);
        if (valid) {
            mc_event ev;
            ev.work = T.work_prefix[p] + (work_of(C, j.view, j.hist) - C.work_begin);
            ev.bin = j.bin_lo;
            ev.emit_voxel = j.voxel;
            ev.weight = w;
            stage[ev_count + lanes_below(m)] = ev;
        }
        ev_count += (uint32_t)__popcll(m);
    }
}

// Set up the n (<= 64) forced copies at the head of a wave's ring and append
// those that score to the wave's job queue (all 64 lanes call).  Most copies
// of collisions score nothing (their energy leaves the window), so their ray
// walks are deferred and run 64 scoring jobs at a time (fd_walk_jobs)
// instead of a few lanes of each drained batch.
template <int MODE>
__device__ inline void fd_drain(const Cst& C, int p, const FdPoint* ring, uint32_t& head, uint32_t n,
                                int lane, const TransportArgs& T, FdJob* jq, uint32_t& jq_tail) {
    wave_sync_lds();
    FdJob j;
    bool ok = false;
    if ((uint32_t)lane < n) {
        const FdPoint q = ring[(head + (uint32_t)lane) & (FD_RING - 1)];
        ok = fd_setup_mode<MODE>(C, T.descs + p, q, j);
    }
    const uint64_t m = __ballot(ok);
    if (ok) jq[(jq_tail + lanes_below(m)) & (FD_JOBS - 1)] = j;
    jq_tail += (uint32_t)__popcll(m);
    head += n;
}

// Walk and score the n (<= 64) jobs at the head of the wave's job queue
// (all 64 lanes call).
template <int MODE>
__device__ inline void fd_walk_jobs(const Cst& C, int p, const FdJob* jq, uint32_t& jq_head, uint32_t n,
                                    int lane, const TransportArgs& T, uint32_t& rays, uint32_t& pieces,
                                    mc_event* stage, uint32_t& ev_count) {
    wave_sync_lds();
    const bool valid = (uint32_t)lane < n;
    FdJob j = {};
    if (valid) j = jq[(jq_head + (uint32_t)lane) & (FD_JOBS - 1)];
    fd_score<MODE>(C, p, j, valid, lane, T, rays, pieces, stage, ev_count);
    jq_head += n;
}

// Persistent transport: waves claim chunks of work until none are left.
// A wavefront emits the next 64 x emit_per_lane histories of its chunk in one
// converged phase into LDS; idle lanes then start histories from there, so
// the per-lane loop only alternates tentative collisions and Kahn attempts.
// MODE 0: analog arrivals into the tally; 1: forced detection (tally);
// 2: convolution-based forced detection (depth layers); 3: weighted analog
// (forced direction and / or forced interaction; arrivals add their weight).
template <int MODE>
__device__ __forceinline__ void transport_body(TransportArgs T, EmitRec* __restrict__ my,
                                               uint32_t* __restrict__ my_pal,
                                               FdPoint* __restrict__ ring,
                                               FdJob* __restrict__ jq,
                                               mc_event* __restrict__ ev_stage) {
    constexpr int EPL = emit_per_lane(MODE);
    constexpr int EBATCH = 64 * EPL;
    // analog: two records of the emission loop at a time, so their table
    // gathers overlap (the weighted kernel measured slower unrolled)
    constexpr int EMIT_UNROLL = MODE == 0 ? 2 : 1;
    constexpr bool FD = MODE == 1 || MODE == 2;
    constexpr bool VR = MODE == 3;
    const bool vr_dir = VR && (T.vr_flags & VR_FORCED_DIRECTION);
    const bool vr_fi = VR && (T.vr_flags & VR_FORCED_INTERACTION);
    const bool count_tallied = !FD && T.n_events && !T.events;
    const int lane = threadIdx.x & 63;
    uint32_t fd_head = 0, fd_tail = 0;    // wave-uniform ring cursors (FD)
    uint32_t jq_head = 0, jq_tail = 0;    // wave-uniform job queue cursors (FD)
    const uint64_t full = __ballot(1);   // lanes of this wavefront
    // chunk bookkeeping (wave-uniform): problem-local work range [c_next, c_end)
    // and the (view, history id) of c_next; staged records [s_next, s_end)
    uint64_t c_next = 0, c_end = 0, cur_view = 0, cur_hist = 0;
    uint32_t s_next = 0, s_end = 0;
    int p = -1;
    bool exhausted = false, have_pending = false;
    uint64_t pending = 0;
    uint32_t fc[7] = {0, 0, 0, 0, 0, 0, 0};   // wave-uniform fate counts
    // packed per-lane fate counts (fold_fates), cheaper per iteration than
    // seven ballots; the weighted mode keeps the ballots (its registers are
    // tighter: the packed counts spill there)
    constexpr bool PACK_FATES = !VR;
    uint64_t fpk = 0;
    uint32_t fpk_iter = 0;
    long long e_esc = 0;                      // escaped energy, Q40.23 (per lane)
    uint32_t fd_rays = 0, fd_pieces = 0;      // forced-copy ray walks, voxels visited (per lane)
    uint32_t ev_count = 0;                    // staged events (forced detection, wave-uniform)
    const bool fd_list = FD && T.events;
    Cst C;
    Lane L;
    L.state = S_IDLE;
    Acc A;            // advance()'s per-lane work counters, summed over the wave at flush
    acc_zero(A);
    // chunk prefix lives after the work prefix: [n_problems + 1] entries
    const uint64_t* __restrict__ chunk_prefix = T.work_prefix + (T.n_problems + 1);
    const uint64_t n_chunks = chunk_prefix[T.n_problems];

    MC_REGION(-1);
    for (;;) {
        MC_REGION(RG_LOOP);
        // Refill: at most one chunk claim and one emission phase per iteration;
        // idle lanes not served wait for the next one.  Lanes only pick a
        // staged slot here and load it below, outside any loop.
        const uint64_t need = __ballot(L.state == S_IDLE);
        int slot = -1;
        if (need != 0 && !exhausted) {
            MC_REGION(RG_REFILL);
            bool ready = true;
            if (s_next >= s_end) {
                // stage empty: emit the next batch of the chunk (claim one if needed)
                if (c_next >= c_end) {
                    if (!have_pending) {
                        unsigned long long base = 0;
                        if (lane == 0) base = atomicAdd(&T.state->next_chunk, 1ull);
                        pending = uniform64(base);
                        have_pending = true;
                        if (pending >= n_chunks) exhausted = true;
                    }
                    if (!exhausted) {
                        // problem of the pending chunk (uniform binary search)
                        int lo = 0, hi = T.n_problems - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (chunk_prefix[mid] <= pending) lo = mid; else hi = mid - 1;
                        }
                        const int np = __builtin_amdgcn_readfirstlane(lo);
                        // drain problem p first: no lane busy, no forced copy queued
                        if (np != p && (need != full || (FD && (fd_tail != fd_head || jq_tail != jq_head)))) {
                            ready = false;                 // drain problem p first
                        } else {
                            if (np != p) {
                                if (p >= 0) {
                                    if (PACK_FATES) fold_fates(fpk, fc);
                                    flush(e_esc, fc, A, fd_rays, fd_pieces, p, T, lane, count_tallied);
                                }
                                p = np;
                                C = load_cst(T.descs + p);
                                if (C.use_pal) {
                                    // the wave is drained: no lane reads the old palette
#pragma unroll
                                    for (int k = 0; k < PALETTE_N / 64; ++k)
                                        my_pal[k * 64 + lane] = ldg(C.pal + k * 64 + lane);
                                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                                    __builtin_amdgcn_wave_barrier();
                                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                                }
                            }
                            const uint64_t local_chunk = pending - chunk_prefix[p];
                            const uint64_t cnt = T.work_prefix[p + 1] - T.work_prefix[p];
                            c_next = local_chunk * T.chunk;
                            c_end = min(c_next + T.chunk, cnt);
                            have_pending = false;
                            if (C.flags != 0) c_next = c_end;   // staging found bad input: skip
                            else split_work(C, C.work_begin + c_next, cur_view, cur_hist);
                        }
                    } else {
                        ready = false;
                    }
                }
                if (ready && c_next < c_end) {
                    MC_REGION(RG_EMIT);
                    const uint32_t n_rec = (uint32_t)min((uint64_t)EBATCH, c_end - c_next);
                    if (fd_list && ev_count > EV_STAGE - EBATCH) flush_events(T, ev_stage, ev_count, lane);
#pragma unroll EMIT_UNROLL
                    for (int k = 0; k < EPL; ++k) {
                        const uint32_t idx = (uint32_t)(k * 64 + lane);
                        FdPoint q = {};
                        if (idx < n_rec) {
                            uint64_t v = cur_view, h = cur_hist;
                            advance_cursor(C, v, h, idx, C.n_views);
                            const Emission e = emit_history(C, (uint32_t)h, (uint32_t)v, vr_dir, T.vr_omc);
                            EmitRec r;
                            r.x = e.x; r.y = e.y; r.z = e.z; r.dx = e.dx; r.dy = e.dy; r.dz = e.dz;
                            r.voxel = e.voxel; r.view = (uint32_t)v; r.hist = (uint32_t)h;
                            const float2 cs = ldg(C.views + v);
                            r.vc = cs.x; r.vs = cs.y;
                            my[idx] = r;
                            if constexpr (FD) {
                                q.x = e.x; q.y = e.y; q.z = e.z;
                                q.e = C.e0;
                                q.view = (uint32_t)v; q.hist = (uint32_t)h; q.event = 0;
                                q.voxel = e.voxel;
                            }
                        }
                        // the emission point's forced copy, scored at once (all
                        // lanes: the event stage is appended wave-wide)
                        if constexpr (FD) {
                            FdJob j;
                            const bool ok = idx < n_rec && fd_setup_mode<MODE>(C, T.descs + p, q, j);
                            fd_score<MODE>(C, p, j, ok, lane, T, fd_rays, fd_pieces, ev_stage, ev_count);
                        }
                    }
                    // the records are read by other lanes of this wavefront
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    s_next = 0;
                    s_end = __builtin_amdgcn_readfirstlane(n_rec);
                    c_next += n_rec;
                    advance_cursor(C, cur_view, cur_hist, n_rec, C.n_views);
                }
            }
            if (ready && s_next < s_end) {
                const uint32_t avail = s_end - s_next;
                const uint32_t rank = lanes_below(need);
                if (L.state == S_IDLE && rank < avail) slot = (int)(s_next + rank);
                // read back as uniform: the cursor then stays in a scalar
                // register and the slot pick above is scalar work
                s_next = __builtin_amdgcn_readfirstlane(s_next + min((uint32_t)__popcll(need), avail));
            }
        }
        if (slot >= 0) {
            MC_REGION(RG_BEGIN);
            const EmitRec r = my[slot];
            Emission e;
            e.x = r.x; e.y = r.y; e.z = r.z; e.dx = r.dx; e.dy = r.dy; e.dz = r.dz;
            e.voxel = r.voxel;
            begin_history(C, L, r.view, r.hist, e);
            L.vc = r.vc; L.vs = r.vs;     // staged: no global load at the history's start
            if (vr_dir) L.w = 0.5f * T.vr_omc;     // Omega / (4 pi)
        }
        MC_REGION(RG_EXIT_TEST);
        if (exhausted && __ballot(L.state != S_IDLE) == 0 && (!FD || (fd_tail == fd_head && jq_tail == jq_head)))
            break;

        int fate = R_RUNNING;
        int iu, iv;               // set by the escape of a history that arrives
        const int before = L.state;
        if (before != S_IDLE) {
            MC_REGION(RG_PHILOX);
            uint32_t c0 = L.hist, c1 = (uint32_t)L.view, c2, c3;
            counter_of(L, c2, c3);
            philox10(c0, c1, c2, c3, C.seed, C.pid);
            fate = advance(C, my_pal, L, c0, c1, c2, c3, A, iu, iv, vr_fi);
            if (fate != R_RUNNING) {
                MC_REGION(RG_FATE_ENERGY);
                // outgoing energy: escaped, or left at the step cap (rare: booked at once)
                const float out = ((fate == MC_ABSORBED) | (fate == MC_CUT)) ? 0.0f : L.e;
                if (fate == MC_CAPPED_FATE) {
                    if (T.energy)
                        atomicAdd((unsigned long long*)(T.energy + (size_t)p * 4 + 2),
                                  (unsigned long long)to_q23(out));
                } else {
                    // Q40.23 as to_q23, zero-extended: the energy is never negative
                    e_esc += (long long)(uint32_t)__float2int_rn(out * 8388608.0f);
                }
            }
        }
        MC_REGION(RG_WORK_COUNT);
        if constexpr (FD) {
            // a real collision: absorbed, or a Compton scatter started
            const bool real = (before == S_STEP) &
                              ((fate == MC_ABSORBED) | ((fate == R_RUNNING) & (L.state == S_KAHN)));
            // real collisions queue their forced copies (position, direction
            // and energy before the collision are still the lane's)
            const uint64_t m = __ballot(real);
            if (m != 0) {
                if (real) {
                    FdPoint q;
                    q.x = L.x; q.y = L.y; q.z = L.z; q.dx = L.dx; q.dy = L.dy; q.dz = L.dz;
                    q.e = L.e; q.view = (uint32_t)L.view; q.hist = L.hist; q.event = L.n;
                    q.voxel = L.emit_voxel;
                    ring[(fd_tail + lanes_below(m)) & (FD_RING - 1)] = q;
                }
                fd_tail += (uint32_t)__popcll(m);
            }
            // the one place forced copies of collisions are scored (one code
            // path, so a score never depends on where it was drained): set
            // up 64 at a time, or what is left once no lane is busy; the
            // walks of those that score run 64 at a time, or the rest once
            // no lane is busy and no copy is queued
            MC_REGION(RG_FORCED);
            const uint32_t cnt = fd_tail - fd_head;
            const bool none_busy = __ballot(L.state != S_IDLE) == 0;
            if (cnt >= 64 || (cnt != 0 && none_busy))
                fd_drain<MODE>(C, p, ring, fd_head, cnt < 64 ? cnt : 64u, lane, T, jq, jq_tail);
            const uint32_t nj = jq_tail - jq_head;
            if (nj >= 64 || (nj != 0 && none_busy && fd_tail == fd_head)) {
                if (fd_list && ev_count > EV_STAGE - 64) flush_events(T, ev_stage, ev_count, lane);
                fd_walk_jobs<MODE>(C, p, jq, jq_head, nj < 64 ? nj : 64u, lane, T, fd_rays, fd_pieces,
                                   ev_stage, ev_count);
            }
        }
        if (__ballot(fate != R_RUNNING) != 0) {
            MC_REGION(RG_FATES);
            if constexpr (PACK_FATES) {
                if (fate != R_RUNNING) fpk += 1ull << (9 * fate);
            } else {
#pragma unroll
                for (int f = 0; f < 7; ++f) fc[f] += (uint32_t)__popcll(__ballot(fate == f));
            }
            const uint64_t tallied = FD ? 0ull : __ballot(fate == MC_TALLIED);
            if (tallied != 0) {
                MC_REGION(RG_TALLY);
                // arrivals: bin, weight (Q31.32) and squared weight (Q31.32 for
                // unit weights, Q11.52 for weighted arrivals)
                uint32_t bin = 0;
                long long w = 0, w2 = 0;
                if (fate == MC_TALLIED) {
                    const int cls = L.n_scatter > 0 ? 1 : 0;
                    bin = (uint32_t)((((uint32_t)L.view * 2u + cls) * (uint32_t)C.nv + iv) * (uint32_t)C.nu + iu);
                    w = signed_weight(T.descs + p, L.emit_voxel,
                                      VR ? __float2ll_rn(L.w * 4294967296.0f) : 1ll << 32);
                    w2 = VR ? __float2ll_rn(L.w * L.w * 4503599627370496.0f) : 1ll << 32;
                }
                if constexpr (VR) {
                    // weighted runs (forced direction) tally most histories, in
                    // bins that are nearly all distinct within a wavefront: one
                    // atomic per lane (the matching loop took 0.99 against 0.75 ms)
                    if (fate == MC_TALLIED) {
                        atomicAdd((unsigned long long*)(T.tally + C.tally_offset + bin), (unsigned long long)w);
                        if (T.tally_sq)
                            atomicAdd((unsigned long long*)(T.tally_sq + C.tally_offset + bin),
                                      (unsigned long long)w2);
                    }
                } else {
                    tally_aggregated(T, C.tally_offset, tallied, bin, w, w2, lane);
                }
                if (T.events) {       // without a list the count is the flushed fate count
                    // one reservation for the wave's arrivals, then one record per lane
                    unsigned long long base = 0;
                    if (lane == 0) base = atomicAdd(T.n_events, (unsigned long long)__popcll(tallied));
                    base = uniform64(base);
                    const unsigned long long idx = base + (unsigned long long)lanes_below(tallied);
                    if (fate == MC_TALLIED && idx < T.event_capacity) {
                        mc_event ev;
                        ev.work = T.work_prefix[p] + (work_of(C, L.view, L.hist) - C.work_begin);
                        ev.bin = bin;
                        ev.emit_voxel = L.emit_voxel;
                        ev.weight = w;
                        T.events[idx] = ev;
                    }
                }
            }
            if (fate != R_RUNNING) L.state = S_IDLE;
        }
        if (PACK_FATES && ++fpk_iter == FATE_FOLD) {
            fold_fates(fpk, fc);
            fpk_iter = 0;
        }
    }
    if (PACK_FATES) fold_fates(fpk, fc);
    if (p >= 0) flush(e_esc, fc, A, fd_rays, fd_pieces, p, T, lane, count_tallied);
    if (fd_list) flush_events(T, ev_stage, ev_count, lane);
    MC_REGION(-2);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_transport(TransportArgs T) {
    __shared__ EmitRec stage[WAVES_PER_BLOCK_MAX][EMIT_BATCH];
    __shared__ uint32_t pal_copy[WAVES_PER_BLOCK_MAX][PALETTE_N];
    transport_body<0>(T, stage[threadIdx.x >> 6], pal_copy[threadIdx.x >> 6], nullptr, nullptr, nullptr);
}

__global__ __launch_bounds__(256) void k_transport_fd(TransportArgs T) {
    __shared__ EmitRec stage[WAVES_PER_BLOCK_MAX][64 * emit_per_lane(1)];
    __shared__ uint32_t pal_copy[WAVES_PER_BLOCK_MAX][PALETTE_N];
    __shared__ FdPoint ring[WAVES_PER_BLOCK_MAX][FD_RING];
    __shared__ FdJob jobs[WAVES_PER_BLOCK_MAX][FD_JOBS];
    __shared__ mc_event ev_stage[WAVES_PER_BLOCK_MAX][EV_STAGE];
    transport_body<1>(T, stage[threadIdx.x >> 6], pal_copy[threadIdx.x >> 6],
                      ring[threadIdx.x >> 6], jobs[threadIdx.x >> 6], ev_stage[threadIdx.x >> 6]);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_transport_vr(TransportArgs T) {
    __shared__ EmitRec stage[WAVES_PER_BLOCK_MAX][EMIT_BATCH];
    __shared__ uint32_t pal_copy[WAVES_PER_BLOCK_MAX][PALETTE_N];
    transport_body<3>(T, stage[threadIdx.x >> 6], pal_copy[threadIdx.x >> 6], nullptr, nullptr, nullptr);
}

__global__ __launch_bounds__(256) void k_transport_cfd(TransportArgs T) {
    __shared__ EmitRec stage[WAVES_PER_BLOCK_MAX][64 * emit_per_lane(2)];
    __shared__ uint32_t pal_copy[WAVES_PER_BLOCK_MAX][PALETTE_N];
    __shared__ FdPoint ring[WAVES_PER_BLOCK_MAX][FD_RING];
    __shared__ FdJob jobs[WAVES_PER_BLOCK_MAX][FD_JOBS];
    transport_body<2>(T, stage[threadIdx.x >> 6], pal_copy[threadIdx.x >> 6],
                      ring[threadIdx.x >> 6], jobs[threadIdx.x >> 6], nullptr);
}

// Replay: one listed history per lane, run to its end, one record out.
__global__ __launch_bounds__(256) void k_replay(const ProbDesc* __restrict__ d,
                                                const int32_t* __restrict__ views,
                                                const uint64_t* __restrict__ hists, int64_t n,
                                                mc_record* __restrict__ out, int32_t vr_flags,
                                                float vr_omc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Cst C = load_cst(d);
    if (i >= n) return;
    Lane L;
    L.hist = (uint32_t)hists[i];
    L.view = views[i];
    L.n = 0; L.n_scatter = 0; L.emit_voxel = 0;
    L.e = 0.0f;
    const bool view_ok = L.view >= 0 && L.view < d->n_views && hists[i] <= 0xFFFFFFFFull;
    Acc A;
    acc_zero(A);
    mc_record r;
    r.fate = -1; r.iu = -1; r.iv = -1;
    if (C.flags == 0 && view_ok) {
        const Emission e = emit_history(C, (uint32_t)L.hist, (uint32_t)L.view,
                                        (vr_flags & VR_FORCED_DIRECTION) != 0, vr_omc);
        begin_history(C, L, (uint32_t)L.view, (uint32_t)L.hist, e);
        for (;;) {
            uint32_t c0 = (uint32_t)L.hist, c1 = (uint32_t)L.view, c2, c3;
            counter_of(L, c2, c3);
            philox10(c0, c1, c2, c3, C.seed, C.pid);
            int iu = -1, iv = -1;
            const int fate = advance(C, C.pal, L, c0, c1, c2, c3, A, iu, iv,
                                     (vr_flags & VR_FORCED_INTERACTION) != 0);
            if (fate != R_RUNNING) {
                r.fate = fate;
                r.iu = iu;
                r.iv = iv;
                break;
            }
        }
    }
    r.view = L.view;
    r.n_scatter = L.n_scatter;
    r.n_tent = (int32_t)A.n_tent;
    r.emit_voxel = (int32_t)L.emit_voxel;
    r.cls = L.n_scatter > 0 ? 1 : 0;
    r.e_final = (double)L.e;
    out[i] = r;
}

// Per-call preparation: zero outputs and counters, work and chunk prefixes.
__global__ __launch_bounds__(256) void k_prepare(const ProbDesc* __restrict__ descs, int n_problems,
                                                 uint64_t* work_prefix, uint32_t chunk,
                                                 CallState* state, int64_t* status,
                                                 unsigned long long* n_events,
                                                 int64_t* tally, uint64_t tally_elems,
                                                 int64_t* tally_sq, int64_t* fates, int64_t* energy,
                                                 int64_t* counters) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = tid; i < tally_elems; i += stride) {
        tally[i] = 0;
        if (tally_sq) tally_sq[i] = 0;
    }
    for (uint64_t i = tid; i < (uint64_t)n_problems * MC_N_FATES; i += stride) fates[i] = 0;
    for (uint64_t i = tid; i < (uint64_t)n_problems * 4; i += stride)
        if (energy) energy[i] = 0;
    for (uint64_t i = tid; i < (uint64_t)n_problems * MC_N_COUNTERS; i += stride)
        if (counters) counters[i] = 0;
    if (tid == 0) {
        uint64_t w = 0, c = 0;
        uint64_t* chunk_prefix = work_prefix + (n_problems + 1);
        for (int p = 0; p < n_problems; ++p) {
            work_prefix[p] = w;
            chunk_prefix[p] = c;
            const uint64_t cnt = descs[p].work_count;
            w += cnt;
            c += (cnt + chunk - 1) / chunk;
        }
        work_prefix[n_problems] = w;
        chunk_prefix[n_problems] = c;
        state->next_chunk = 0;
        status[0] = 0; status[1] = 0; status[2] = 0; status[3] = 0;
        if (n_events) *n_events = 0;
    }
}

// After transport: fold staging flags and list overflow into status.
__global__ void k_finalize(const ProbDesc* __restrict__ descs, int n_problems, int64_t* status,
                           const unsigned long long* n_events, uint64_t capacity,
                           const int64_t* fates, int64_t* energy) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint64_t f = 0;
    int64_t n_pal = 0;
    for (int p = 0; p < n_problems; ++p) {
        f |= descs[p].flags;
        n_pal += descs[p].pal_state == 0;
        if (energy) {
            // every history started at the line energy: what did not leave
            // (escaped or capped) was deposited
            int64_t nh = 0;
            for (int k = 0; k < MC_N_FATES; ++k) nh += fates[(size_t)p * MC_N_FATES + k];
            int64_t* e = energy + (size_t)p * 4;
            e[0] = nh * (int64_t)llrint((double)descs[p].e0 * 8388608.0) - e[1] - e[2];
        }
    }
    if (n_events && capacity != UINT64_MAX && *n_events > capacity) f |= MC_STATUS_LIST_OVERFLOW;
    status[0] |= (int64_t)f;
    status[2] = n_pal;
}

// Tally range check, TALLY_CHECK_BLOCKS workgroups per problem.  A source
// of one sign adds weights of one sign (at most 2^32 each), so a bin that
// crossed 2^63 reads negative: any negative bin is an overflow.  A
// difference source adds both signs; its analog bins stay in range while
// fewer than 2^31 histories are tallied in all (each adds +-2^32), which is
// what is checked for it (its forced-detection and weighted forms are not
// checked: each history then scores up to one weight per collision).
constexpr int TALLY_CHECK_BLOCKS = 128;   // ~16 elements per thread on a 60-view 64x64 tally

__global__ __launch_bounds__(256) void k_tally_check(const ProbDesc* __restrict__ descs,
                                                     const int64_t* __restrict__ tally,
                                                     const int64_t* __restrict__ fates,
                                                     int64_t* status) {
    const int p = blockIdx.x / TALLY_CHECK_BLOCKS, part = blockIdx.x % TALLY_CHECK_BLOCKS;
    const ProbDesc& d = descs[p];
    bool bad = false;
    if (d.act_prev) {
        bad = part == 0 && threadIdx.x == 0 && fates[(size_t)p * MC_N_FATES + MC_TALLIED] >= (1ll << 31);
    } else {
        const uint64_t n = (uint64_t)d.n_views * 2u * (uint64_t)d.nv * (uint64_t)d.nu;
        const int64_t* t = tally + d.tally_offset;
#pragma unroll 4
        for (uint64_t i = (uint64_t)part * 256 + threadIdx.x; i < n; i += TALLY_CHECK_BLOCKS * 256)
            bad |= t[i] < 0;
    }
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0)
        atomicOr((unsigned long long*)status, (unsigned long long)MC_STATUS_TALLY_OVERFLOW);
}

__global__ void k_zero_status(int64_t* status) {
    if (blockIdx.x == 0 && threadIdx.x < 4) status[threadIdx.x] = 0;
}

}  // namespace

hipError_t launch_prepare_call(const ProbDesc* descs, int32_t n_problems, uint64_t* work_prefix,
                               CallState* state, int64_t* status, unsigned long long* n_events,
                               int64_t* tally, uint64_t tally_elems, int64_t* tally_sq,
                               int64_t* fates, int64_t* energy, int64_t* counters, uint32_t chunk,
                               hipStream_t s) {
    uint64_t g = (tally_elems + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    k_prepare<<<(int)g, 256, 0, s>>>(descs, n_problems, work_prefix, chunk, state, status, n_events,
                                     tally, tally_elems, tally_sq, fates, energy, counters);
    return hipGetLastError();
}

hipError_t launch_tally_check(const ProbDesc* d_desc, int n_problems, const int64_t* tally,
                              const int64_t* fates, int64_t* status, hipStream_t s) {
    k_tally_check<<<n_problems * TALLY_CHECK_BLOCKS, 256, 0, s>>>(d_desc, tally, fates, status);
    return hipGetLastError();
}

hipError_t launch_transport(const TransportArgs& a, int grid, int block, hipStream_t s) {
    if (a.vr_flags) k_transport_vr<<<grid, block, 0, s>>>(a);
    else if (a.forced_detection == 2) k_transport_cfd<<<grid, block, 0, s>>>(a);
    else if (a.forced_detection) k_transport_fd<<<grid, block, 0, s>>>(a);
    else k_transport<<<grid, block, 0, s>>>(a);
    // without a list the count is informational and cannot overflow
    k_finalize<<<1, 64, 0, s>>>(a.descs, a.n_problems, a.status, a.n_events,
                                a.events ? a.event_capacity : UINT64_MAX, a.fates, a.energy);
    return hipGetLastError();
}

hipError_t launch_replay(const ProbDesc* d_desc, const int32_t* views, const uint64_t* hists,
                         int64_t n, mc_record* out, int64_t* status, int block, int32_t vr_flags,
                         float vr_omc, hipStream_t s) {
    k_zero_status<<<1, 64, 0, s>>>(status);
    if (n > 0) {
        const int64_t g = (n + block - 1) / block;
        k_replay<<<(int)g, block, 0, s>>>(d_desc, views, hists, n, out, vr_flags, vr_omc);
    }
    k_finalize<<<1, 64, 0, s>>>(d_desc, 1, status, nullptr, 0, nullptr, nullptr);
    return hipGetLastError();
}

int transport_blocks_per_cu(int block, int forced_detection, int vr_flags) {
    int n = 0;
    const hipError_t e = vr_flags
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_transport_vr, block, 0)
        : forced_detection == 2
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_transport_cfd, block, 0)
        : forced_detection
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_transport_fd, block, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_transport, block, 0);
    if (e != hipSuccess) return 1;
    return n > 0 ? n : 1;
}

}  // namespace mcs

#ifdef MC_REGION_PROFILE
// Measurement build only: copy the region totals of the transport loop
// (entries and shader-clock cycles, RG_COUNT + 1 values each; the last is the
// time before the first marker) to host arrays, or zero them (reset != 0).
extern "C" int mc_region_profile(unsigned long long* counts, unsigned long long* cycles, int reset) {
    using namespace mcs;
    const size_t nb = sizeof(unsigned long long) * RG_SLOTS;
    if (reset) {
        unsigned long long z[RG_SLOTS] = {0};
        hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_region_count), z, nb);
        if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(g_region_cycles), z, nb);
        return (int)e;
    }
    if (!counts || !cycles) return MC_EINVAL;
    hipError_t e = hipMemcpyFromSymbol(counts, HIP_SYMBOL(g_region_count), nb);
    if (e == hipSuccess) e = hipMemcpyFromSymbol(cycles, HIP_SYMBOL(g_region_cycles), nb);
    return (int)e;
}
#endif
