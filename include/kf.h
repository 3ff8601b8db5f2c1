/*
 * kf.h -- C ABI of the MI355X batched Kalman-filter track fitter (libkfmi.so).
 *
 * The library fits many independent charged-particle tracks at once.  Each
 * track is a list of hits on planes, discs, cylinders (2-D hits) or straws
 * (lines: 1-D hits, the drift distance).  The fit is the Kalman-filter
 * track fit of the paper (Sect. 2, Fig. 1): adaptive Runge-Kutta-Nystrom
 * propagation from surface to surface with the transport Jacobian and the
 * local<->global Jacobians (Sect. 4.1), a gain-matrix update on every measured
 * surface (Sect. 2, step 3), then a Rauch-Tung-Striebel smoother that reuses
 * the Jacobians stored during the forward pass (Sect. 2, smoother paragraph),
 * or, on request, the paper's other smoother: a second Kalman filter run
 * backwards and combined with the forward one (Sect. 2, Fig. 2).
 * The matrix inverse the smoother needs is always done in FP64 (Sect. 4.2.4).
 * The field is uniform, solenoid-like or a tabulated map; the fitted
 * parameters come on the seed surface or at the perigee of a line.
 * The per-track data sets follow Sect. 4.3: measurements, starting
 * parameters, fit configuration (target surface), and results (status,
 * track states, fitted parameters at the target surface).
 *
 * Conventions
 *   units            mm, GeV, T, ns, rad
 *   bound parameters (loc0, loc1, phi, theta, q/p, t) -- Sect. 2 parameter list;
 *                    phi in (-pi, pi], theta in [0, pi]
 *   covariances      packed upper triangle, row-major: (0,0),(0,1)..(0,5),(1,1)..(5,5)
 *   surfaces         planes with centre c and rotation R = [u v n] (columns);
 *                    loc0 = u.(r - c), loc1 = v.(r - c); surfaces are unbounded;
 *                    a disc (kf_surfaces.type) measures the polar coordinates of
 *                    (u.(r - c), v.(r - c)) instead; a cylinder (axis through c
 *                    along n) the position along the axis and the azimuth about
 *                    it; a line (straw: wire through c along n) the signed
 *                    distance of closest approach to the wire
 *   array layout     component-major ("[3][S]" means 3 rows of S items); every
 *                    array pointer is a DEVICE pointer owned by the caller
 *   hits             CSR over tracks: hits of track t are hit_offsets[t] ..
 *                    hit_offsets[t+1]-1, in the order the track crosses them
 *   seed surface     the starting parameters live on one plane (kf_seeds);
 *                    the fitted parameters are returned on that same surface
 *                    (it is the fit's target surface) unless kf_config.target
 *                    asks for the perigee
 *
 * Execution: every entry point validates its arguments on the host before any
 * device work, then enqueues kernels on `stream` (a hipStream_t, NULL = the
 * null stream) and returns without waiting.  Inputs must stay valid until the
 * stream reaches the work.  The library allocates no device memory: the
 * caller passes a workspace of at least kf_workspace_bytes().  Calls that
 * share a workspace must not overlap.
 *
 * Errors: a negative return is an argument error found on the host before any
 * launch (nothing was enqueued), or KF_E_HIP if the HIP runtime refused a
 * launch.  Per-track problems are reported in status[t] (KF_ST_*); a failed
 * track's outputs are NaN and never affect other tracks.
 */
#ifndef KF_H
#define KF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define KF_OK 0
#define KF_E_NULL (-1)      /* a required pointer is NULL */
#define KF_E_SIZE (-2)      /* a count is negative, too large, or inconsistent */
#define KF_E_ENUM (-3)      /* an enum field has an unknown value */
#define KF_E_WS (-4)        /* workspace missing or too small */
#define KF_E_HIP (-5)       /* the HIP runtime reported an error */
#define KF_E_VALUE (-6)     /* a configuration value is out of range (tolerance <= 0, ...), or the
                               workgroup size needs more LDS than the device has for this
                               surface count (14 doubles per surface + 14.5 KiB per 64 threads) */
#define KF_E_SCRATCH (-7)   /* kf_fit_tracks_noalloc: the batch needs more workspace than the
                               library's static scratch (KF_NOALLOC_SCRATCH_BYTES) */

/* ---- per-track status ---- */
#define KF_ST_OK 0
#define KF_ST_NO_INTERSECT 1   /* direction parallel to a target plane (|n.T| < 1e-6) */
#define KF_ST_STEP_CAP 2       /* more than max_steps RKN trials in one gap */
#define KF_ST_NOT_SPD 3        /* residual covariance or predicted covariance not positive definite */
#define KF_ST_BAD_INPUT 4      /* non-finite input, non-SPD hit or seed covariance, bad surface id,
                                  or more hits than kf_measurements.max_hits */
#define KF_ST_TOO_FEW 5        /* fewer than 3 hits */

/* ---- enums ---- */
#define KF_FIELD_UNIFORM 0     /* B = b0 everywhere */
#define KF_FIELD_SOLENOID 1    /* Bz = b0[2] (1 - a z^2), Bx = a b0[2] x z, By = a b0[2] y z */
#define KF_FIELD_MAP 2         /* tabulated: trilinear interpolation in kf_field.map */

#define KF_PREC_FP64 0         /* every step in FP64 */
#define KF_PREC_MIXED 1        /* RKN stepping and transport Jacobian in FP32 on increments
                                  from an FP64 anchor; landing, update, smoother in FP64 */

#define KF_SCHED_AUTO 0        /* pick from the autotune table */
#define KF_SCHED_DIRECT 1      /* one lane per track, tracks in input order */
#define KF_SCHED_SORTED 2      /* tracks sorted by hit count (longest first), persistent waves
                                  pull 64-track tiles from a queue */

#define KF_JAC_STORE 0         /* transport Jacobians stored by the filter, read by the smoother */
#define KF_JAC_RECOMPUTE 1     /* smoother re-propagates the filtered state (less memory traffic) */

#define KF_OUT_AUTO 0          /* from the autotune table, else STAGED */
#define KF_OUT_STAGED 1        /* RTS: the wave's smoothed states are staged in LDS and written to the
                                  outputs every two smoother steps (no round trip through the
                                  workspace) */
#define KF_OUT_SLOTS 2         /* RTS: each smoothed state replaces its hit's prediction in the
                                  workspace; a tile's outputs are then written four hits at a time
                                  (longer runs per track, one more workspace round trip).  The two
                                  paths give the same outputs bit for bit; the two-filter smoother
                                  always writes through its slots */

#define KF_SMOOTHER_RTS 0         /* Rauch-Tung-Striebel with the forward pass's transport Jacobians */
#define KF_SMOOTHER_TWO_FILTER 1  /* a second Kalman filter from the last hit back to the seed surface,
                                     propagating against the direction of flight, combined with the
                                     forward filter (Sect. 2, Fig. 2) */

#define KF_TARGET_SEED_SURFACE 0  /* tgt_par / tgt_cov on the seed surface */
#define KF_TARGET_PERIGEE 1       /* tgt_par / tgt_cov at the perigee of a line parallel to z */

#define KF_SURF_PLANE 0        /* local (u.(r - c), v.(r - c)) */
#define KF_SURF_DISC 1         /* local polar (|d|, atan2(v.d, u.d)), d = (u.(r - c), v.(r - c)): radius
                                  and azimuth about the centre in the surface's plane */
#define KF_SURF_CYLINDER 2     /* axis through c along n, radius rho (kf_surfaces.radius): local
                                  (n.(r - c), atan2(v.(r - c), u.(r - c))), position along the axis and
                                  azimuth; r = c + rho (cos l1 u + sin l1 v) + l0 n.  The landing is the
                                  crossing where the track moves outward (the larger root of the
                                  straight-line distance to go) */
#define KF_SURF_LINE 3         /* straw: wire through c along n; loc0 = e.(r - c), e = (n x T)/|n x T|,
                                  the signed distance of closest approach (the only measured
                                  coordinate: a 1-D hit, loc[1] and cov[1..2] are not read), loc1 =
                                  n.(r - c) along the wire.  The landing is the closest approach
                                  (Newton steps on (r - c)_perp . T = 0); the material is crossed across
                                  the wire (path x/X0 / |n x T|) */

#define KF_MAX_SURFACES 512     /* the surface table is staged in LDS (14 doubles each) */
#define KF_MAX_HITS 64         /* per track */

typedef struct {
    int32_t n;                 /* number of surfaces S (1 .. KF_MAX_SURFACES) */
    const double *center;      /* [3][S] */
    const double *rot;         /* [9][S] row-major 3x3, columns u, v, n (orthonormal) */
    const double *x_over_X0;   /* [S] material thickness in radiation lengths (0 = none) */
    const double *align;       /* [6][S] optional (NULL = none): alignment correction per surface,
                                  (dx, dy, dz, alpha, beta, gamma); the fit uses the surface with
                                  centre c + (dx, dy, dz) and rotation R Rx(alpha) Ry(beta) Rz(gamma)
                                  (turned about its own u, v, n axes) */
    const int32_t *type;       /* [S] optional (NULL = all planes): KF_SURF_* per surface.  The seed
                                  surface must be a plane and every hit's surface a plane or a disc,
                                  or, with `radius` given, also a cylinder (radius > 0) or a line
                                  (else that track gets KF_ST_BAD_INPUT).  On a disc or a cylinder
                                  the measured azimuth, its residual and the filtered and smoothed
                                  azimuths are taken in (-pi, pi].  kf_fit_tracks_vjp requires NULL */
    const double *radius;      /* [S] optional: cylinder radii (mm; read for KF_SURF_CYLINDER only).
                                  Give it (any values for other types) to fit cylinders and lines:
                                  with type and radius set the fit runs the kernels built for every
                                  surface type, one wave per SIMD (kf_config.occupancy 0 or 1; others
                                  give KF_E_VALUE).  NULL: types 2 and 3 are unknown types.
                                  kf_fit_tracks_vjp requires NULL */
} kf_surfaces;

typedef struct {
    int32_t kind;              /* KF_FIELD_* */
    double b0[3];              /* T (UNIFORM, SOLENOID) */
    double a;                  /* 1/mm^2, KF_FIELD_SOLENOID only */
    /* KF_FIELD_MAP (Sect. 4.1: position-dependent field information kept in
     * memory): B at the grid points map_origin + (i, j, k) * map_spacing,
     * 0 <= i < map_n[0] etc. (each >= 2, spacing > 0), interpolated
     * trilinearly in the cell that holds the point, with the interpolant's
     * gradient for the transport Jacobian.  A coordinate outside the grid is
     * clamped to its boundary (the field there is the boundary's; no
     * gradient along that axis). */
    int32_t map_n[3];
    double map_origin[3];      /* mm */
    double map_spacing[3];     /* mm */
    const double *map;         /* device pointer, [map_n[2]][map_n[1]][map_n[0]][3] (Bx, By, Bz in T);
                                  read by the kernels, owned by the caller */
} kf_field;

typedef struct {
    int32_t n_tracks;          /* N >= 0 */
    int32_t max_hits;          /* upper bound of hits per track (1 .. KF_MAX_HITS); tracks with
                                  more hits get KF_ST_BAD_INPUT */
    int64_t n_hits;            /* H = hit_offsets[N] (the host cannot read device memory) */
    const int32_t *hit_offsets;  /* [N+1] non-decreasing, hit_offsets[0] = 0 */
    const int32_t *surface_id;   /* [H] */
    const double *loc;           /* [2][H] measured loc0, loc1 */
    const double *cov;           /* [3][H] hit covariance v00, v01, v11 */
} kf_measurements;

typedef struct {
    const double *par;         /* [6][N] starting parameters on the seed surface */
    const double *cov;         /* [21][N] their covariance (the prior), packed upper */
    int32_t surface_id;        /* the seed / target surface */
} kf_seeds;

typedef struct {
    int32_t precision;           /* KF_PREC_* */
    int32_t multiple_scattering; /* 1: thin-scatterer process noise after each update (Highland) */
    double mass;                 /* GeV */
    double rk_tol;               /* RKN local error tolerance [mm], e.g. 1e-4 */
    double land_tol;             /* landing tolerance on the distance to a plane [mm], e.g. 1e-6; the
                                    remaining distance is covered by a second-order move */
    int32_t max_steps;           /* RKN trials per gap, e.g. 1000 */
    int32_t schedule;            /* KF_SCHED_* */
    int32_t block;               /* threads per workgroup (64, 128, 256), 0 = autotuned */
    int32_t waves_per_cu;        /* persistent schedule: resident waves per CU, 0 = autotuned */
    int32_t occupancy;           /* register budget as waves per SIMD (1, 2, 3), 0 = autotuned */
    int32_t split_smoother;      /* 0: smoother in the same kernel as the filter; 1: separate kernel */
    int32_t jacobians;           /* KF_JAC_STORE: the filter stores each transport Jacobian for the
                                    smoother (52 workspace doubles per hit); KF_JAC_RECOMPUTE: the
                                    smoother propagates each filtered state again instead (27 doubles
                                    per hit; fused smoother only) */
    int32_t smoother;            /* KF_SMOOTHER_*.  TWO_FILTER: the backward filter starts at the last
                                    hit from the forward filtered state there with its covariance times
                                    bwd_scale, and takes in every hit on its way back; at each surface
                                    it adds the scatterer's variance as the forward filter evaluated it
                                    (at the forward filtered state) after propagating back, and its
                                    prediction (hits after k) combines with the forward filtered state
                                    (hits up to k): K = Cf (Cf + Cb)^-1, xs = xf + K (xb - xf),
                                    Cs = (I - K) Cf (I - K)^T + K Cb K^T.  The last hit keeps its
                                    filtered state; the seed surface gets the combination with the
                                    seed.  Fused smoother only (split_smoother 0; jacobians ignored);
                                    kf_fit_tracks_vjp supports RTS only */
    double bwd_scale;            /* TWO_FILTER: inflation of the backward filter's starting covariance
                                    (> 1; 0 = 1e3).  Its information, 1/bwd_scale of the last
                                    filtered state's, counts twice in the combination */
    int32_t target;              /* KF_TARGET_*.  PERIGEE (Sect. 2; Sect. 5.2): the fitted state on
                                    the seed surface is propagated (FP64, whatever the precision) to
                                    the closest approach to the line through `perigee` parallel to
                                    z and given as (d0, z0, phi, theta, q/p, t): d0 = (r - c) . u with
                                    u = (-sin phi, cos phi, 0), z0 = r_z - c_z; the covariance goes
                                    with that transport's Jacobian.  A track whose perigee is not
                                    reached (|T_perp| too small, or more than max_steps trials) gets
                                    KF_ST_NO_INTERSECT / KF_ST_STEP_CAP and NaN outputs.
                                    kf_fit_tracks_vjp supports the seed surface only */
    double perigee[3];           /* PERIGEE: a point c of the line (mm) */
    int32_t output;              /* KF_OUT_*: how the RTS smoother's states reach the outputs */
} kf_config;

typedef struct {
    double *par;               /* [6][H] smoothed parameters at every hit */
    double *cov;               /* [21][H] smoothed covariance at every hit */
    double *tgt_par;           /* [6][N] fitted parameters on the seed/target surface */
    double *tgt_cov;           /* [21][N] */
    double *chi2;              /* [N] sum of predicted-residual chi2 increments */
    int32_t *ndf;              /* [N] measured coordinates (2 per hit, 1 on a line) less 5 with field,
                                  less 4 without */
    uint8_t *status;           /* [N] KF_ST_* */
    int32_t *trials;           /* [H] optional (NULL): RKN trials taken to reach each hit */
    double *filt_par;          /* [6][H] optional (NULL): filtered parameters */
    double *filt_cov;          /* [21][H] optional (NULL) */
} kf_outputs;

/* Library version string (static storage). */
const char *kf_version(void);

/* Text for a return code or (if code >= 0) a per-track status. */
const char *kf_status_string(int code);

/* Bytes of workspace kf_fit_tracks needs for these sizes (0 on bad arguments).
 * Grows as n_tracks * max_hits * 52 doubles (predicted state and covariance and
 * transport Jacobian per hit) plus small per-track and per-tile tables. */
size_t kf_workspace_bytes(const kf_config *cfg, const kf_measurements *meas, int32_t n_surfaces);

/* Filter + smoother (RTS or two-filter, cfg->smoother) for every track
 * (Sect. 2; Sect. 4.1; Sect. 4.3).
 * All pointers inside the structs are device pointers except where stated.
 * Returns KF_OK or a negative KF_E_* code; per-track results in out->status. */
int kf_fit_tracks(const kf_config *cfg, const kf_surfaces *surf, const kf_field *field,
                  const kf_measurements *meas, const kf_seeds *seeds, const kf_outputs *out,
                  void *workspace, size_t workspace_bytes, void *stream);

/* A captured fit: the whole launch sequence of kf_fit_tracks (length sort +
 * fit kernels) for one fixed set of arguments and buffers, recorded once into
 * a HIP graph and replayed by kf_plan_launch.  The arrays the arguments point
 * to must stay allocated (their contents may change) until kf_plan_destroy.
 * AUTO settings are resolved at creation.  Launches of one plan must not
 * overlap (they share the workspace). */
typedef struct kf_plan kf_plan;

int kf_plan_create(const kf_config *cfg, const kf_surfaces *surf, const kf_field *field,
                   const kf_measurements *meas, const kf_seeds *seeds, const kf_outputs *out,
                   void *workspace, size_t workspace_bytes, kf_plan **plan);
int kf_plan_launch(kf_plan *plan, void *stream);
void kf_plan_destroy(kf_plan *plan);

/* Launch-shape autotuner (the paper's grid/block/register studies, Sect. 5.3,
 * made automatic): times every candidate schedule (direct / length-sorted
 * persistent), workgroup size, register budget (waves per SIMD), fused or
 * separate smoother kernel, stored or recomputed transport Jacobians, the
 * output path (RTS only: a two-filter fit tries the fused kernel alone; a
 * fixed cfg->output is kept) and
 * persistent waves per CU on these very buffers
 * (outputs are overwritten), synchronising `stream`.  Writes the fastest
 * setting to *best (and its time per fit to *best_ms if not NULL) and
 * remembers it: later calls with AUTO (0) settings and the same precision,
 * field kind, smoother, surface kinds (with or without cylinders and lines),
 * max_hits and track count (to a power of two) use it. */
int kf_autotune(const kf_config *cfg, const kf_surfaces *surf, const kf_field *field,
                const kf_measurements *meas, const kf_seeds *seeds, const kf_outputs *out,
                void *workspace, size_t workspace_bytes, void *stream, kf_config *best, float *best_ms);

/* ---- fit without a caller workspace and without allocation ----
 *
 * For callers that cannot allocate device memory at all (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * kf_fit_tracks_noalloc runs exactly the fit of kf_fit_tracks (same kernels,
 * same launch settings, same results bit for bit) but takes its workspace
 * from a static device array of KF_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on, until the process ends.  It calls no
 * hipMalloc, hipFree or other allocating routine.  The scratch of the current
 * device is used; `stream` must belong to that device.  Its address is looked
 * up once per device, on the first call made with that device current.
 * Batches whose kf_workspace_bytes() exceeds KF_NOALLOC_SCRATCH_BYTES are
 * refused with KF_E_SCRATCH before anything is enqueued (64 MiB holds e.g.
 * 16,000 tracks of 10 hits or 5,000 tracks of 30 hits).  All calls on one
 * device share the one array: calls whose work overlaps on the device race
 * (serialise them, e.g. on one stream).  What must start at zero (the
 * length-sort counters) is cleared by a kernel of every call; the rest is
 * written before it is read.  Other arguments and return codes as
 * kf_fit_tracks. */
#define KF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int kf_fit_tracks_noalloc(const kf_config *cfg, const kf_surfaces *surf, const kf_field *field,
                          const kf_measurements *meas, const kf_seeds *seeds, const kf_outputs *out,
                          void *stream);

/* ---- fit from host memory, copies overlapped with the fit ----
 *
 * The paper's timeline (Sect. 5.3) counts the host <-> device transfers next
 * to the kernel (about 17 % of the run time with one stream; overlapping them
 * with several streams is limited by the transfer time).  kf_fit_tracks_staged
 * takes the measurements, seeds and outputs in HOST memory (surfaces and field
 * as for kf_fit_tracks, in device memory) and cuts the batch into n_chunks
 * ranges of consecutive tracks.  Chunk i runs on streams[i % n_streams]: its
 * inputs are copied in (rows of the component-major arrays as 2D copies), its
 * CSR offsets rebased on the device, the fit of kf_fit_tracks is enqueued on
 * them, and the outputs are copied back; with n_streams >= 2 the copies of one
 * chunk overlap the fit of another.  Results are those of kf_fit_tracks on the
 * whole batch, bit for bit (tracks are independent).  Host buffers must stay
 * valid until the streams are synchronised and should be pinned (page-locked,
 * e.g. hipHostMalloc), otherwise the copies do not overlap.  The optional
 * outputs (trials, filtered states) are not supported: they must be NULL.
 * cfg launch settings resolve per chunk as for kf_fit_tracks.  Streams must
 * not be NULL; the library synchronises nothing.  Returns KF_E_VALUE for
 * n_chunks < 1 or n_streams < 1 (n_chunks above n_tracks is clamped).
 *
 * Workspace: n_streams slots, each with device buffers for one chunk's
 * inputs, outputs and fit workspace, sized for the largest chunk. */
size_t kf_staged_workspace_bytes(const kf_config *cfg, const kf_measurements *host_meas, int32_t n_surfaces,
                                 int32_t n_chunks, int32_t n_streams);
int kf_fit_tracks_staged(const kf_config *cfg, const kf_surfaces *surf, const kf_field *field,
                         const kf_measurements *host_meas, const kf_seeds *host_seeds,
                         const kf_outputs *host_out, void *workspace, size_t workspace_bytes,
                         int32_t n_chunks, void *const *streams, int32_t n_streams);

/* ---- adjoint (vector-Jacobian product) of the fit ----
 *
 * For the scalar L = sum_t g_chi2[t] chi2_t + sum_hits g_par . (smoothed
 * parameters) + sum_t g_tgt . (fitted parameters on the target surface),
 * kf_fit_tracks_vjp returns dL/d(measured loc0, loc1) of every hit, dL/d(the
 * alignment correction) of every surface and, optionally, dL/d(starting
 * parameters) of every track.  It is the reverse of the whole fit: the RTS
 * smoother (Sect. 2), the gain-matrix update, the covariance transport and the
 * adaptive RKN propagation with its transport Jacobian (Sect. 4.1), including
 * the dependence of that Jacobian on the state.  The forward fit is recomputed
 * per track (nothing from an earlier kf_fit_tracks call is reused); the
 * propagation of each gap is replayed with the forward pass's own step
 * decisions and reversed step by step (stages, transport-Jacobian columns,
 * step sizes capped at the target plane, landing, local <-> global maps), so
 * the gradient is that of the discrete fit the forward call computes.  The
 * precision follows cfg->precision: with KF_PREC_FP64 every step is FP64;
 * with KF_PREC_MIXED the forward recompute and the replay of each gap step in
 * FP32 on the FP64 anchor exactly as the mixed fit does (same states, same
 * step decisions), and everything else -- the reverse sweep through the
 * steps, evaluated at the replayed states, the update, covariance and
 * smoother algebra and every adjoint accumulation -- is FP64.  The alignment
 * gradient of a surface sums over all tracks in a fixed order: the result is
 * bitwise reproducible.  A track whose recomputed fit fails contributes
 * nothing to the alignment gradient and gets NaN in its meas and seed rows. */
typedef struct {
    const double *chi2;        /* [N] dL/dchi2 per track, or NULL (zero) */
    const double *par;         /* [6][H] dL/d(smoothed parameters) per hit, or NULL (zero) */
    const double *tgt_par;     /* [6][N] dL/d(fitted target parameters), or NULL (zero) */
} kf_cotangents;

typedef struct {
    double *meas;              /* [2][H] dL/d(loc0, loc1) per hit (required if H > 0) */
    double *align;             /* [6][S] dL/d(dx, dy, dz, alpha, beta, gamma) per surface at the
                                  surfaces' alignment (kf_surfaces.align, zero if NULL), or NULL */
    double *seed;              /* [6][N] dL/d(starting parameters), or NULL */
    uint8_t *status;           /* [N] status of the recomputed fit (KF_ST_*), or NULL */
} kf_gradients;

/* Workspace bytes for kf_fit_tracks_vjp (0 on bad arguments): n_tracks *
 * max_hits * 87 doubles of per-hit state, 6 doubles per hit and per track of
 * alignment contributions, and the reduction's partial sums. */
size_t kf_vjp_workspace_bytes(const kf_config *cfg, const kf_measurements *meas, int32_t n_surfaces);

/* Enqueue the adjoint.  Arguments as kf_fit_tracks; cfg->schedule and
 * cfg->block select the launch (AUTO: length-sorted persistent schedule).
 * Returns KF_OK or a negative KF_E_* code. */
int kf_fit_tracks_vjp(const kf_config *cfg, const kf_surfaces *surf, const kf_field *field,
                      const kf_measurements *meas, const kf_seeds *seeds, const kf_cotangents *cot,
                      const kf_gradients *grad, void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KF_H */
