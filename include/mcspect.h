/*
 * mcspect.h -- C ABI of the MI355X Monte Carlo SPECT transport library.
 *
 * The library estimates SPECT projections by following photon histories one by
 * one from emission to absorption, energy cut or escape (paper: Zhou et al.,
 * "Application of Monte Carlo algorithms to cardiac imaging reconstruction",
 * Sec. 2), through a voxelised attenuation map, into a rotating parallel-hole
 * camera with a photopeak energy window (Sec. 3).  Tallied photons give the
 * projections P_j and the Monte Carlo response matrix T_ij of Sec. 5.1,
 * Eq. IMC; mlem_iterate runs the update of Sec. 5.1, Eq. MLEM.
 *
 * Physics model (the paper names none; these are this library's definitions):
 *  - mu_v(E) = mu_v * g(E): every material is density-scaled water;
 *    g(E) = (1-f) sigma_KN(E)/sigma_KN(140) + f (140/E)^3 with f the
 *    photoelectric share of attenuation at 140 keV (pe_fraction);
 *  - Woodcock tracking against mu_max(E) = max_v mu_v * g(E); a tentative
 *    collision in voxel v is real iff (r >> 8) < Q_v, Q_v = ceil(mu_v 2^24 /
 *    max mu) evaluated in double precision;
 *  - photoelectric absorption with probability f (140/E)^3 / g(E), otherwise
 *    Compton scatter with Kahn's Klein-Nishina sampler and uniform azimuth;
 *  - the collimator accepts an escaping photon iff d . n_view >= cos(alpha).
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), key (seed,
 * problem_id), counter (history id, view, event, sub-draw), so every history
 * can be replayed on its own.  Uniforms are ((r >> 9) + 1/2) 2^-23.
 *
 * Geometry: lengths in cm, energies in keV.  The voxel grid [nz][ny][nx]
 * (x fastest) is centred on the origin.  View k has normal n_k = (cos t_k,
 * sin t_k, 0), detector axes u_k = (-sin t_k, cos t_k, 0) and z, and its
 * plane is n_k . p = radius_cm.  N histories split over V views as
 * N_k = floor(N/V) + [k < N mod V], history ids 0..N_k-1 within view k; the
 * work index g runs view-major over (view, history id).
 *
 * Conventions for every entry point:
 *  - Pointers documented "device" are HIP device memory owned by the caller;
 *    "host" pointers are read during the call only.
 *  - Calls are asynchronous on the given stream (hipStream_t passed as void*,
 *    NULL = default stream).  Results are valid after the stream synchronises.
 *  - The library allocates no device memory: scratch comes from the caller's
 *    workspace, sized by the matching *_workspace_bytes function.
 *  - Return value: MC_OK or a negative MC_E* code.  Argument checks that need
 *    device data (negative or NaN mu, zero activity, list overflow, capped
 *    histories) are reported through the device status array instead.
 *  - No C++ exception crosses this interface.  Calls on different streams with
 *    different workspaces may run concurrently.
 */
#ifndef MCSPECT_H
#define MCSPECT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MC_OK = 0,
    MC_EINVAL = -1,     /* invalid argument (host-visible)                    */
    MC_ENOMEM = -2,     /* workspace or output capacity too small             */
    MC_EDEVICE = -3,    /* a HIP call failed; see mc_last_hip_error()         */
    MC_EOVERFLOW = -4,  /* fixed-point overflow (mc_check_status)             */
    MC_ECAPPED = -5     /* some history hit max_steps (mc_check_status)       */
};

/* Bits of status[0] (device int64 written by mc_simulate_projections). */
enum {
    MC_STATUS_BAD_MU = 1,        /* a mu value is negative, NaN or infinite   */
    MC_STATUS_NO_ACTIVITY = 2,   /* activity sums to zero                     */
    MC_STATUS_BAD_ANGLE = 4,     /* a view angle is not finite                */
    MC_STATUS_LIST_OVERFLOW = 8, /* more tallied histories than list_capacity */
    MC_STATUS_CAPPED = 16,       /* a history hit max_steps (fate CAPPED)     */
    MC_STATUS_GRAD_OVERFLOW = 32,/* a gradient term exceeded the fixed-point  */
                                 /* range at this frac_bits (term dropped)    */
    MC_STATUS_BAD_EVENT = 64,    /* an event did not replay to its bin        */
    MC_STATUS_ACTIVITY_OVERFLOW = 128,/* a block activity sum exceeds 32 bits */
    MC_STATUS_TALLY_OVERFLOW = 256    /* a tally bin may have left Q31.32: a     */
                                      /* negative bin of a source of one sign, or */
                                      /* 2^31 or more tallied histories of a      */
                                      /* difference source (analog)               */
};

enum { MC_N_COUNTERS = 8 };   /* work counters per problem */

/* Fate counters, in this order: */
enum { MC_ABSORBED = 0, MC_CUT = 1, MC_ESCAPED = 2, MC_ESCAPED_FOV = 3,
       MC_OUT_OF_WINDOW = 4, MC_TALLIED = 5, MC_CAPPED_FATE = 6, MC_N_FATES = 8 };

/* Emission modes. */
enum { MC_SOURCE_VOXELS = 0,   /* voxel by activity, uniform inside it          */
       MC_SOURCE_POINT = 1 };  /* grid centre exactly (voxel still drawn)       */

typedef struct {
    int32_t nx, ny, nz;         /* grid size                                    */
    int32_t source_mode;        /* MC_SOURCE_*                                  */
    double voxel_cm;            /* cubic voxel edge                             */
    const float* mu140;         /* device [nz*ny*nx], 1/cm at 140 keV           */
    const uint32_t* activity;   /* device [nz*ny*nx], integer emission weights  */
    int32_t n_views;            /* V >= 1                                       */
    int32_t nu, nv;             /* detector bins along u and z                  */
    const double* angle_rad;    /* device [n_views], view angles                */
    double pixel_cm;            /* square detector bin edge                     */
    double radius_cm;           /* detector plane distance from the axis        */
    double accept_half_angle_rad; /* collimator cone half-angle, (0, pi/2)      */
    double e_lo_kev, e_hi_kev;  /* photopeak window, closed interval            */
    double e_cut_kev;           /* photons below this energy are cut            */
    double pe_fraction;         /* photoelectric share of attenuation at 140 keV*/
    uint64_t n_histories;       /* N, defines the split over views              */
    uint64_t history_offset;    /* first work index simulated by this call      */
    uint64_t history_count;     /* work indices simulated (0 = to the end)      */
    uint32_t seed, problem_id;  /* Philox key                                   */
    int32_t image_factor;       /* >0: image voxel = phantom voxel / factor     */
    uint32_t max_steps;         /* cap on tentative collisions (0 = 1000)       */
    const uint32_t* activity_prev; /* device [nz*ny*nx] or NULL: reuse of photon */
                                /* tracks (Sec. 5.3): the source is then the    */
                                /* signed difference d = activity -             */
                                /* activity_prev; histories are drawn from |d|  */
                                /* and every tally contribution (and event      */
                                /* weight) carries the sign of d at the         */
                                /* emitting voxel, so tally x sum|d| / (N / V)  */
                                /* is the projection of d, to be added to that  */
                                /* of activity_prev.  Forward projection only:  */
                                /* mc_adjoint_mu and mc_system_matrix reject it */
    double e0_kev;              /* emission line energy (Sec. 3: Tc-99m 140,    */
                                /* Tl-201 71 and 167 keV); 0 = 140.  At most    */
                                /* 500 keV, exactly representable in FP32, and  */
                                /* >= e_cut_kev.  mu140 stays the map at 140    */
                                /* keV (scaled by g(E)).  A multi-line source   */
                                /* is one problem per line (histories split by  */
                                /* the line intensities); problems with the     */
                                /* same seed and problem_id run the same        */
                                /* histories, so a line tallied in several      */
                                /* windows is several problems differing only   */
                                /* in e_lo_kev / e_hi_kev                       */
} mc_problem;

typedef struct {
    int32_t hist_per_lane;      /* histories per lane per work claim, <=0: auto */
    int32_t block_size;         /* threads per block (64..256), <=0: auto       */
    int32_t blocks_per_cu;      /* resident blocks per CU to launch, <=0: auto  */
    int32_t brick_log2;         /* accept-threshold layout: 0 linear (default), */
                                /* 2 or 3: 4^3 or 8^3 voxel bricks              */
    int32_t threshold_bytes;    /* bytes per voxel of the threshold table: 0 or */
                                /* 1: one-byte codes into a 256-entry palette   */
                                /* when the map has at most 256 distinct        */
                                /* thresholds (else 4); 4: always 32-bit        */
    int32_t forced_detection;   /* mc_simulate_projections only: 1 = the tally  */
                                /* is the forced-detection estimate (Sec. 5.2)  */
                                /* instead of analog arrivals; 2 = convolution- */
                                /* based forced detection; 0 = analog; also     */
                                /* passed to mc_workspace_bytes (2 needs more)  */
    void* kernel_events[2];     /* optional hipEvent_t pair recorded on the     */
                                /* stream right before / after the transport    */
                                /* kernel (NULL: none)                          */
    int32_t variance_reduction; /* weighted analog transport (Sec. 5.2), bits:  */
                                /* 1 forced direction: every photon leaves in   */
                                /* the cone of the half-angle below about the   */
                                /* view normal (the same two emission words),   */
                                /* weight (1 - cos) / 2; 2 forced interaction:  */
                                /* a real collision is always Compton and the   */
                                /* weight takes 1 - p_pe(E).  Arrivals add     */
                                /* their weight (Q31.32) to the tally and its   */
                                /* square (Q11.52) to tally_sq, and events      */
                                /* carry it.  Not with forced_detection; the    */
                                /* adjoint rejects it; replay honours it.       */
    int32_t pad_vr;
    double forced_direction_half_angle_rad;  /* (0, pi] when bit 1 is set      */
    int32_t reuse_staging;      /* mc_adjoint_mu only: 1 = the workspace holds  */
                                /* the staged tables of this same problem, with */
                                /* unchanged inputs, from the last              */
                                /* mc_simulate_projections that used it (one    */
                                /* problem, earlier on the same stream): the    */
                                /* staging passes are skipped                   */
    int32_t pad_rs;
} mc_options;

/* One tally contribution, as written to the optional event list: a tallied
 * history (analog), or one forced-detection score. */
typedef struct {
    uint64_t work;        /* call-global work index (problems concatenated)     */
    uint32_t bin;         /* bin within its problem: ((view*2+cls)*nv+iv)*nu+iu */
    uint32_t emit_voxel;  /* phantom voxel of emission                          */
    int64_t weight;       /* contribution to the bin, Q31.32: 1 << 32 for an    */
                          /* analog arrival, the score for a forced copy        */
} mc_event;

/* Per-history record written by mc_replay_histories. */
typedef struct {
    int32_t fate, view, iu, iv;   /* iu = iv = -1 when no detector bin        */
    int32_t n_scatter, n_tent;    /* Compton scatters, tentative collisions   */
    int32_t emit_voxel, cls;      /* cls 0 primary, 1 scattered (tallied)     */
    double e_final;               /* energy at the end of the history (keV)   */
} mc_record;

/* Bytes of workspace that mc_simulate_projections / mc_replay_histories /
 * mc_adjoint_mu need for these problems.  Returns 0 on invalid arguments. */
size_t mc_workspace_bytes(const mc_problem* problems, int32_t n_problems,
                          const mc_options* opt);

/* Forward Monte Carlo projection of n_problems phantoms in one persistent
 * launch (Sec. 2 transport, Sec. 3 camera; the projections P_j of Eq. IMC).
 *   problems   host [n_problems]
 *   opt        host, nullable (defaults)
 *   tally      device int64 [sum_p V_p*2*nv_p*nu_p], Q31.32 fixed point sum of
 *              weights, layout [problem][view][class][iv][iu]; overwritten
 *   tally_sq   device, same shape, sum of squared weights; nullable
 *   fates      device int64 [n_problems][8]; overwritten
 *   energy     device int64 [n_problems][4], Q40.23 keV: deposited, escaped,
 *              capped, 0; nullable
 *   counters   device int64 [n_problems][MC_N_COUNTERS]: tentative
 *              collisions, real collisions, Kahn attempts, histories, then
 *              (forced detection) the forced copies whose ray was walked to
 *              the detector and the voxels those walks visited, 0, 0;
 *              nullable
 *   events     device mc_event [event_capacity], tallied histories in no
 *              particular order; nullable
 *   n_events   device uint64 [1], number of tallied histories (may exceed the
 *              capacity: then status has MC_STATUS_LIST_OVERFLOW); nullable
 *   status     device int64 [4]: [0] MC_STATUS_* bits, [1] capped histories,
 *              [2] problems whose thresholds were read as one-byte palette
 *              codes (see mc_options.threshold_bytes)
 *   workspace  device, at least mc_workspace_bytes(...)
 * Results are bit-identical from run to run and independent of the options
 * (apart from forced_detection, which changes what the tally estimates).
 *
 * Forced detection (opt->forced_detection = 1; Sec. 5.2): the analog
 * histories run unchanged (fates, energies and counters are theirs), but the
 * tally is scored by forced copies: at each history's emission point (class
 * 0) and at each real collision (class 1) a copy leaves in a direction drawn
 * uniformly in the collimator cone (Philox event of the point, sub-draw
 * 0x80000000) with weight Omega_cone * pdf * exp(-g(E') * integral of mu140
 * along the ray to the grid edge), pdf = 1/(4 pi) at emission and
 * (1 - p_pe(E)) times the Klein-Nishina angular density at a collision; no
 * score when E' is cut, outside the window or the ray misses the detector.
 * The expected score of every bin equals its expected analog count.  The
 * tally stays Q31.32; tally_sq holds the sum of squared scores in Q11.52.
 * The event list, if given, holds one event per nonzero score (its weight is
 * the score; n_events counts them), so mc_system_matrix builds the forced-
 * detection response matrix from it; without a list n_events stays 0.
 *
 * Convolution-based forced detection (opt->forced_detection = 2; Sec. 5.2):
 * the same histories and forced copies, but each copy goes along the detector
 * normal n_k with the weight above taken at that direction, and is stored in
 * the depth layer l = floor((D - n_k . x) / pixel) (clamped to the
 * ceil(2 D / pixel) layers) at the pixel of its perpendicular hit.  After
 * transport every layer is convolved with the response of the ideal cone
 * collimator at its centre depth d = (l + 1/2) pixel: the plane density of
 * directions uniform in the cone, d / (2 pi (1 - cos a) (d^2 + r^2)^(3/2))
 * for r <= d tan a, integrated over each pixel with 8 x 8 midpoint samples
 * and normalised, on offsets -h..h with h = ceil(d tan a / pixel + 1/2); the
 * convolved layers (FP64, rounded once to Q31.32) are the tally.  tally_sq
 * stays 0, events must be NULL (MC_EINVAL otherwise) and n_events stays 0.
 * Problems whose deepest response has h > 24 are rejected (MC_EINVAL); the
 * workspace holds the layers, 8 * V * L * 2 * nv * nu bytes per problem.
 * mc_adjoint_mu takes analog event lists only. */
int mc_simulate_projections(const mc_problem* problems, int32_t n_problems,
                            const mc_options* opt,
                            int64_t* tally, int64_t* tally_sq, int64_t* fates,
                            int64_t* energy, int64_t* counters,
                            mc_event* events, uint64_t event_capacity, uint64_t* n_events,
                            int64_t* status,
                            void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and arguments as mc_simulate_projections, without a workspace.
 * The scratch comes from one array of MC_STATIC_SCRATCH_BYTES (64 MiB) per
 * device, placed in device memory when the library's code is loaded and held
 * until the process ends; the call allocates nothing.  Problems whose
 * mc_workspace_bytes exceed it are refused with MC_ENOMEM (a 128^3 grid
 * fits).  Every call on a device shares that device's array: calls that
 * overlap on one device (different streams, threads) race and must be
 * serialised by the caller.  The outputs are the caller's, as for
 * mc_simulate_projections, and are bit-identical to its. */
#define MC_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
int mc_simulate_projections_static(const mc_problem* problems, int32_t n_problems,
                                   const mc_options* opt,
                                   int64_t* tally, int64_t* tally_sq, int64_t* fates,
                                   int64_t* energy, int64_t* counters,
                                   mc_event* events, uint64_t event_capacity, uint64_t* n_events,
                                   int64_t* status, void* stream);

/* Re-run the listed histories of problem 0 one per lane and write one record
 * each (the replay contract: a history is a function of its Philox counter).
 *   views, hists   device [n]: view and history id of each history
 *   records        device mc_record [n]                                     */
int mc_replay_histories(const mc_problem* problem, const mc_options* opt,
                        const int32_t* views, const uint64_t* hists, int64_t n,
                        mc_record* records, int64_t* status,
                        void* workspace, size_t workspace_bytes, void* stream);

/* Gradient of sum_b G_b * tally_b with respect to mu140 (the adjoint of the
 * forward projection), by path-frozen likelihood ratios: each tallied history
 * is replayed from its Philox counter and its path walked voxel by voxel,
 *   dL/dmu_v = sum_h G_{b(h)} * (c_{h,v} / mu_v - sum_seg g(E_seg) len(seg, v)),
 * c_{h,v} = Compton vertices of h in v.  Only tallied histories contribute.
 *   problem     host, the same description as the forward call
 *   dL_dtally   device double [V*2*nv*nu], G in the tally layout
 *   events      device, the forward call's event list (replay just those), or
 *               NULL to replay every history of the range
 *   n_events    device uint64 [1], the forward call's count (read on device)
 *   event_capacity  the list's capacity (host)
 *   dL_dmu      device int64 [nz*ny*nx], overwritten: fixed point with
 *               frac_bits (0..62) fractional bits; value = dL_dmu * 2^-frac_bits
 *   status      device int64 [4]: MC_STATUS_* bits in [0]
 * The sum is exact integer arithmetic: bit-identical from run to run. */
int mc_adjoint_mu(const mc_problem* problem, const mc_options* opt, const double* dL_dtally,
                  const mc_event* events, const uint64_t* n_events, uint64_t event_capacity,
                  int64_t* dL_dmu, int32_t frac_bits, int64_t* status,
                  void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes of mc_system_matrix (0 on invalid arguments): about 36 B
 * per event of capacity (radix-sort buffers) plus 8 B per bin and voxel. */
size_t mc_system_matrix_workspace_bytes(const mc_problem* problem, uint64_t event_capacity);

/* Monte Carlo response matrix of Sec. 5.1 (Eq. IMC) from a forward call's
 * event list: T_ij = c_ij / n_i(j), the estimated probability that a photon
 * emitted in image voxel i is counted in projection bin j; c_ij sums the
 * weights of the events emitted in i and counted in j (the number of tallied
 * histories for an analog list, forced-detection scores for a forced-
 * detection list), n_i(j) = N_view(j) A_i / A
 * the expected emissions from i towards bin j's view (A_i: activity of image
 * voxel i, A: total).  Image voxel = phantom voxel / image_factor per axis
 * (image_factor >= 1).  Bins merge the primary and scatter classes:
 * j = (view * nv + iv) * nu + iu, n_bins = V nv nu.  Both orientations are
 * written as CSR with columns ascending:
 *   T_rowptr   device int64 [n_bins + 1];  T_col int32, T_val float [capacity]
 *   Tt_rowptr  device int64 [n_img + 1];   Tt_col int32, Tt_val float [capacity]
 *   proj       device float [n_bins]: P_j = sum_i c_ij (nullable)
 * c_ij is summed in Q31.32 integers, so the result does not depend on the
 * order of the list.
 * nnz = T_rowptr[n_bins] = Tt_rowptr[n_img] <= min(*n_events, capacity).
 * A list that lost events (*n_events > capacity, read on the device) gives
 * no matrix: every value of T_val, Tt_val and proj is written as NaN (the
 * Python binding reads the count and raises instead).  The forward call must
 * have covered the whole work range (history_offset 0, history_count 0 or
 * n_histories): N_view is the view's share of n_histories; MC_EINVAL
 * otherwise.
 * events / n_events / event_capacity: as returned by mc_simulate_projections
 * for this problem.  class_mask selects the tallied histories used: bit 0
 * primaries, bit 1 scattered photons (3: all; 1: the primary-only matrix a
 * dual-matrix or additive-scatter reconstruction backprojects with; 2: with
 * proj, the scatter projection).  Deterministic (integer counts, sorted
 * rows). */
int mc_system_matrix(const mc_problem* problem, const mc_event* events, const uint64_t* n_events,
                     uint64_t event_capacity, int32_t class_mask,
                     int64_t* T_rowptr, int32_t* T_col, float* T_val,
                     int64_t* Tt_rowptr, int32_t* Tt_col, float* Tt_val, float* proj,
                     void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes of mlem_iterate. */
size_t mlem_workspace_bytes(int64_t n_bins, int64_t n_vox);

/* n_iter MLEM updates (Sec. 5.1, Eq. MLEM):
 *   S_i <- S_i / sens_i * sum_j T_ij P_j / y_j,  y = T S,  sens_i = sum_j T_ij,
 * with T given as CSR in both orientations (rows = bins: T_*, rows = voxels:
 * Tt_*, the same matrix), float values, double accumulation.  image: device
 * float [n_vox], in: S^0 (voxels with sens_i = 0 are set to 0), out: S^n_iter.
 * proj: device float [n_bins].  A bin with y_j = 0 contributes nothing.
 * nnz: the entry count, T_rowptr[n_bins] = Tt_rowptr[n_vox], as the caller
 * knows it from building the matrix; it picks the layout and schedule before
 * launch, and is checked on the device: a different value leaves the image
 * NaN.  Each iteration sweeps only the non-empty rows of T and T^T (listed
 * once per call): two kernels per iteration.  A sparse matrix (nnz <= n_bins
 * + n_vox) is iterated in a compact layout (vectors over the non-empty rows,
 * columns renumbered once per call) whose gathers stay in L2; on a large
 * detector (n_bins >= 2^19, nnz >= 16 n_vox) the backprojection works on one
 * bin slice per XCD (a third kernel adds the slices); columns of each Tt row
 * in ascending order (as mc_system_matrix writes them) give the slices their
 * locality, any order gives the same result.  Deterministic: the summation
 * order depends only on the matrix.  Asynchronous on stream: no host
 * synchronisation, no allocation, no memset, so a call can be captured in a
 * graph (mc_graph_begin) and replayed. */
int mlem_iterate(int64_t n_bins, int64_t n_vox, int64_t nnz,
                 const int64_t* T_rowptr, const int32_t* T_col, const float* T_val,
                 const int64_t* Tt_rowptr, const int32_t* Tt_col, const float* Tt_val,
                 const float* proj, float* image, int32_t n_iter,
                 void* workspace, size_t workspace_bytes, void* stream);

/* mlem_iterate in two parts, for many reconstructions with one matrix
 * (Sec. 5.1: the matrix is fixed while the image is iterated).
 * mlem_prepare does the matrix's share once: the sensitivities sum_j T_ij,
 * the lists of non-empty rows, the renumbered columns of the compact layout
 * and the bin slices, all kept in the workspace together with the entry-count
 * check and a fingerprint (n_bins, n_vox, nnz).  mlem_iterate_prepared then
 * runs n_iter updates exactly as mlem_iterate does (same results bit for
 * bit) without repeating that set-up: the arguments are mlem_iterate's, and
 * the matrix (structure and values) must be the one prepared in this
 * workspace, which must not be used for another matrix in between.  A call
 * whose sizes or entry count differ from the prepared fingerprint, or on a
 * matrix whose entry check failed, sweeps nothing and leaves the image NaN
 * (a workspace never prepared holds no valid fingerprint only by chance: pass
 * a prepared one).  proj and image may change from call to call.  Both are
 * asynchronous on stream, allocate nothing and can be captured in a graph.
 * Errors: as mlem_iterate (mlem_prepare takes no proj, image or n_iter). */
int mlem_prepare(int64_t n_bins, int64_t n_vox, int64_t nnz,
                 const int64_t* T_rowptr, const int32_t* T_col, const float* T_val,
                 const int64_t* Tt_rowptr, const int32_t* Tt_col, const float* Tt_val,
                 void* workspace, size_t workspace_bytes, void* stream);
int mlem_iterate_prepared(int64_t n_bins, int64_t n_vox, int64_t nnz,
                          const int64_t* T_rowptr, const int32_t* T_col, const float* T_val,
                          const int64_t* Tt_rowptr, const int32_t* Tt_col, const float* Tt_val,
                          const float* proj, float* image, int32_t n_iter,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes of osem_iterate (bt_nnz: the entry count of b); 0 for
 * invalid sizes or more than 64 subsets. */
size_t osem_workspace_bytes(int64_t n_bins, int64_t n_vox, int32_t n_subsets, int64_t bt_nnz);

/* Ordered-subsets reconstruction in the forms the paper reviews (Sec. 5.3,
 * Sec. 5.4): OSEM; the dual-matrix update of Eq. DMOS (reproject with c,
 * backproject with b); OS-EM with an additive Monte Carlo scatter projection
 * s (the Sohlberg OS-EM equation).  Subset k holds the views v with
 * v mod n_subsets == k (view of bin j = j / bins_per_view); one iteration
 * visits the subsets in order k = 0..n_subsets-1, each
 *   y_j = sum_i c_ij S_i + s_j            (bins j of subset k)
 *   S_i <- S_i / sens_k,i * sum_{j in k} b_ij P_j / y_j,  sens_k,i = sum_{j in k} b_ij
 * (voxels with sens_k,i = 0 keep their value for that subset; voxels no bin
 * sees start and stay at 0).  n_subsets = 1, b = c, s = NULL is MLEM.
 *   C_*   CSR of c, rows = bins;  Bt_*  CSR of b transposed, rows = voxels
 *   proj  device float [n_bins];  scatter  device float [n_bins] or NULL
 *   bt_nnz the entry count of b, Bt_rowptr[n_vox], as the caller knows it;
 *         checked on the device: a different value leaves the image NaN
 *   image device float [n_vox]: S^0 in, result out.
 * 1 <= n_subsets <= min(64, number of views), else MC_EINVAL.  Once per call
 * B^T is split by subset in the workspace (for subset k and voxel i, the
 * entries of row i whose bin is in subset k, in row order), so each subset's
 * backprojection reads only its own entries.  FP32 matrix values, FP64
 * accumulation.  Column indices must lie in range (C_col < n_vox, Bt_col <
 * n_bins; not checked).  Errors: MC_EINVAL for bad sizes or null pointers,
 * MC_ENOMEM if workspace_bytes < osem_workspace_bytes(...).  Asynchronous on
 * stream, no allocation. */
int osem_iterate(int64_t n_bins, int64_t n_vox, int32_t bins_per_view, int32_t n_subsets,
                 const int64_t* C_rowptr, const int32_t* C_col, const float* C_val,
                 const int64_t* Bt_rowptr, const int32_t* Bt_col, const float* Bt_val, int64_t bt_nnz,
                 const float* proj, const float* scatter, float* image, int32_t n_iter,
                 void* workspace, size_t workspace_bytes, void* stream);

/* Coarse-grid scatter modelling (Sec. 5.4), step 1: the source with larger
 * source voxels.  Every voxel of out takes the summed activity of the
 * f x f x f block holding it, so that the simulator's emission (voxel by
 * activity, uniform inside the voxel) is uniform over the block.
 *   act, out  device uint32 [nz][ny][nx] (distinct buffers)
 *   status    device int64 [1]: MC_STATUS_ACTIVITY_OVERFLOW is or-ed in if a
 *             block sum exceeds 2^32 - 1 (that block is written saturated)
 * nx, ny, nz must be multiples of f >= 1 (MC_EINVAL otherwise).  The coarse
 * problem is the same problem with activity = out, nu / f by nv / f
 * detector bins of f times the pixel size. */
int mc_block_activity(const uint32_t* act, int32_t nx, int32_t ny, int32_t nz, int32_t factor,
                      uint32_t* out, int64_t* status, void* stream);

/* Coarse-grid scatter modelling (Sec. 5.4), step 2: a projection simulated
 * on the coarse detector, expanded and interpolated to the normal pixels:
 * out pixel (j, i) of every plane = the bilinear interpolation at
 * ((i + 1/2) / f - 1/2, (j + 1/2) / f - 1/2) in coarse pixel units (each
 * coordinate clamped to [0, n_c - 1]) of the coarse values read as samples
 * at the coarse pixel centres, divided by f^2 (counts per normal pixel),
 * times scale (1 for counts; A V / N for activity units, as mc_scale_tally).
 *   coarse  device int64 [n_planes][nv_c][nu_c], Q31.32 (a tally: planes =
 *           views x classes)
 *   out     device double [n_planes][nv_c f][nu_c f]
 * MC_EINVAL for sizes < 1 or a non-finite scale. */
int mc_expand_projection(const int64_t* coarse, int64_t n_planes, int32_t nu_c, int32_t nv_c,
                         int32_t factor, double scale, double* out, void* stream);

/* Total weight of a source (Sec. 5.3): sum over the n_vox voxels of
 * |activity - activity_prev| (of activity when activity_prev is NULL), the
 * number a reuse-of-photon-tracks projector sets its histories by.
 *   activity, activity_prev  device uint32 [n_vox] (activity_prev nullable)
 *   total                    device uint64 [1], overwritten (exact)
 * MC_EINVAL for n_vox < 1 or a NULL activity / total. */
int mc_source_total(const uint32_t* activity, const uint32_t* activity_prev, int64_t n_vox,
                    uint64_t* total, void* stream);

/* A Q31.32 tally in activity units (Sec. 5.3, Sec. 5.4): out[i] = tally[i]
 * 2^-32 scale, or out[i] + tally[i] 2^-32 scale when accumulate = 1 -- the
 * projection of the new estimate as the old projection plus the scaled
 * projection of the difference source (reuse of photon tracks; scale = A V /
 * N for a source of total weight A simulated with N histories over V views).
 *   tally  device int64 [n];  out  device double [n]
 * MC_EINVAL for n < 1, a non-finite scale or accumulate not 0 or 1. */
int mc_scale_tally(const int64_t* tally, int64_t n, double scale, double* out, int32_t accumulate,
                   void* stream);

/* Graph capture of a fixed sequence of library calls (the batched launch,
 * response-matrix builds, reconstruction), for callers that replay it:
 * mc_graph_begin starts capturing `stream` (thread-local capture mode); the
 * calls then enqueued on it are recorded, not run; mc_graph_end ends the
 * capture and instantiates it; mc_graph_launch replays it on a stream;
 * mc_graph_destroy frees it.  The calls keep the pointers, sizes and options
 * they were given at capture.  The library's kernels clear their outputs and
 * counters themselves (no memset nodes), so every replay recomputes from the
 * inputs.  stream must not be NULL (the legacy default stream cannot be
 * captured). */
typedef struct mc_graph_s* mc_graph;
int mc_graph_begin(void* stream);
int mc_graph_end(void* stream, mc_graph* graph);
int mc_graph_launch(mc_graph graph, void* stream);
int mc_graph_destroy(mc_graph graph);

/* Launch options for a set of problems (the autotuner of the batched launch):
 * for each of n_candidates option sets, one untimed mc_simulate_projections
 * and reps timed ones (HIP events around the transport kernel); *best
 * receives the index of the fastest (smallest of its reps), times_ms
 * (host, nullable, [n_candidates]) each candidate's best time.  Options only
 * change layout and scheduling (not forced_detection / variance reduction,
 * which change the estimate), so every candidate gives bit-identical
 * outputs; tally, fates and status hold the last run's.  workspace must
 * hold mc_workspace_bytes for these problems.  Synchronous: returns when the
 * last run has finished. */
int mc_autotune(const mc_problem* problems, int32_t n_problems, const mc_options* candidates,
                int32_t n_candidates, int32_t reps, int64_t* tally, int64_t* fates, int64_t* status,
                void* workspace, size_t workspace_bytes, void* stream, int32_t* best, float* times_ms);

/* The outcome a status array records, as a return code (synchronous: waits
 * for `stream`, then reads status[0] from the device):
 *   MC_EINVAL    bad device input (MC_STATUS_BAD_MU, _NO_ACTIVITY,
 *                _BAD_ANGLE, _BAD_EVENT)
 *   MC_EOVERFLOW a fixed-point sum left its range (_GRAD_OVERFLOW,
 *                _TALLY_OVERFLOW, _ACTIVITY_OVERFLOW)
 *   MC_ENOMEM    the event list was too small (_LIST_OVERFLOW)
 *   MC_ECAPPED   some history stopped at max_steps (_CAPPED)
 *   MC_OK        none of these
 * in this order of precedence; MC_EDEVICE if the copy fails.
 *   status  device int64 [>= 1], as written by the calls above */
int mc_check_status(const int64_t* status, void* stream);

/* Human-readable text for an MC_* code (static storage). */
const char* mc_error_string(int code);

/* The last HIP error code seen by this library on the calling thread. */
int mc_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCSPECT_H */
