/*
 * nufft2 -- type-2 NUFFT that evaluates double-Fourier-sphere (DFS) series at
 * semi-Lagrangian departure points, on one AMD Instinct MI355X (gfx950).
 *
 * What is computed (section 5, eq. std_dfs_exp): for every field F and point j
 *
 *     out[F][j] = sum_{n} sum_{m} c[F][n][m] * exp(i (m * phi_j + n * theta_j))
 *
 * with n over the K_theta theta (colatitude) modes and m over the K_phi phi
 * (longitude) modes, centred: coefficient row a holds n = a - K_theta/2 and
 * column b holds m = b - K_phi/2 (integer division).  The sign of the
 * exponent is +i and there is no normalisation.  Section 5 recasts the
 * evaluation as a type-II nonuniform DFT and evaluates it with an NUFFT to
 * a user tolerance eps; this library does the same with three stages:
 *   1. deconvolution by the kernel's Fourier transform and zero padding onto
 *      a 2x upsampled periodic grid,
 *   2. the 2-D inverse FFT of that grid,
 *   3. a w x w "exponential of semicircle" kernel interpolation at each point.
 * Accuracy contract (relative l2 error of a field against the exact sum,
 * at the default kernel width for eps): at most eps for the decaying
 * spectra of smooth fields at general points; up to about 1.5 eps (FP32)
 * and 2.5 eps (FP64, eps >= 1e-12; 3.5 eps below) for flat (white-noise)
 * spectra or for points that sit exactly on fine-grid nodes, where the
 * width rule of the cited method is at its limit (measured: 1.06 eps at
 * w = 7 on grid nodes in exact arithmetic; on flat spectra 1.2 eps at
 * w = 7, 1.6 at w = 9 and 11, 2.35 at w = 13, 2.8 at w = 14, 3.35 at
 * w = 15).  Asking for eps / 10 (one more tap per axis) gives at most eps
 * in every case.
 *
 * Around the interpolation (declared further down):
 *   nufft2_group_*     many plans of uneven size as one unit (an ensemble);
 *   nufft2_autotune    kernel width and gather tiles measured for a problem;
 *   nufft2_server_*    a request loop with continuous batching under an HBM
 *                      budget (host buffers in and out);
 *   nufft2_setpts_vector  setpts with the rotation Q of section 3 applied
 *                      to (u, v) inside every exec;
 *   nufft2_rotate_uv   the same rotation as a separate pass over an output;
 *   nufft2_analysis_*  Grid [0] samples -> exp-form coefficients (section 4),
 *                      with the zonal filter of section 4;
 *   nufft2_pr_*        the partial-regularity expansion of section 4;
 *   nufft2_gl_*        Gauss-Legendre grid samples -> exp-form coefficients
 *                      (section 5, the interpolation for the SHT model).
 *
 * Every entry point returns a status; arguments are checked before anything
 * is enqueued and nothing is enqueued when a call fails.  Work is enqueued on
 * the plan's HIP stream and is asynchronous with respect to the host.  A plan
 * is not thread safe; distinct plans are independent.
 */
#ifndef NUFFT2_H
#define NUFFT2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nufft2_plan_s *nufft2_handle;

typedef enum {
    NUFFT2_OK = 0,
    NUFFT2_ERR_ARG = 1,        /* null pointer, bad size, unsupported shape */
    NUFFT2_ERR_EPS_RANGE = 2,  /* eps below what the precision can reach */
    NUFFT2_ERR_ALLOC = 3,      /* device allocation failed (nothing leaked) */
    NUFFT2_ERR_NO_POINTS = 4,  /* exec before setpts */
    NUFFT2_ERR_NONFINITE = 5,  /* check: a point coordinate was NaN or Inf */
    NUFFT2_ERR_HIP = 6         /* HIP runtime or launch error; see info */
} nufft2_status;

typedef enum { NUFFT2_FP32 = 1, NUFFT2_FP64 = 2 } nufft2_prec;

/* Optional settings; a zero field selects the default. */
typedef struct {
    int32_t w;            /* kernel width in fine-grid cells, 2..16; default from eps */
    double beta_over_w;   /* kernel shape beta / w; default 2.30 */
    int32_t tile_theta;   /* gather tile rows (power of two, 4..128); default 16,
                             8 for FP64 plans with hermitian = 1 */
    int32_t tile_phi;     /* gather tile columns (power of two, 4..128); default 32,
                             64 with hermitian = 1 */
    int32_t real_output;  /* 1: write only the real part (fields known to be real) */
    int32_t hermitian;    /* 1: real fields, see below (implies real output) */
    int32_t m_major;      /* 1: coefficients stored mode-m outer, see nufft2_exec */
    int32_t reserved;     /* 0 */
} nufft2_opts;

typedef struct {
    int32_t prec;          /* nufft2_prec */
    int32_t w;             /* kernel width */
    double beta;           /* kernel shape parameter */
    int64_t n_modes_theta, n_modes_phi;
    int64_t nf_theta, nf_phi;  /* upsampled grid, powers of two >= 2 * modes */
    int32_t n_fields;
    int32_t real_output;
    int32_t tile_theta, tile_phi;
    int64_t n_bins;
    int64_t n_pts;         /* -1 before the first setpts */
    uint64_t workspace_bytes;
    int32_t last_hip_error;  /* hipError_t of the last failure, 0 if none */
    int32_t device;
    int32_t hermitian;       /* 1: real-field plan */
    int32_t fields_per_pass; /* fields the gather stages together: fields f
                                and g share a pass iff f / this == g / this */
    int32_t m_major;         /* 1: coefficients [n_fields][n_modes_phi][n_modes_theta] */
    int32_t reserved;
} nufft2_info;

/*
 * nufft2_plan -- create a plan for n_fields fields of n_modes_theta x
 * n_modes_phi coefficients at tolerance eps.
 *   prec    NUFFT2_FP32: FFT and interpolation in FP32 (coefficients and
 *           output FP32); point coordinates are still wrapped and split in
 *           FP64.  eps >= 1e-7.
 *           NUFFT2_FP64: everything in FP64.  eps >= 1e-15.
 *   The kernel width is w = ceil(log10(1/eps)) + 1 (13 at 1e-12, 7 at 1e-6)
 *   unless opts->w is set.  The fine grid is the smallest power of two
 *   >= max(2 * modes, 2 * w, 32) per dimension and must not exceed 4096.
 *   Real fields (opts->hermitian = 1; both mode counts odd): the
 *   coefficients of a real field satisfy c[-n][-m] = conj(c[n][m])
 *   (section 5, eq. dfs_fourier_coeffs), so the upsampled grid is real and
 *   only the m >= 0 half of the coefficients is needed.  Such a plan reads
 *   coefficient columns K_phi/2 .. K_phi-1 only, transforms them to a real
 *   fine grid (half the data of the complex path through every stage) and
 *   writes real output: for any input it computes
 *       out[F][j] = Re sum_n sum_{m >= 0} (m > 0 ? 2 : 1) c[F][n][m] e^{i (m phi_j + n theta_j)},
 *   which for coefficients of a real field is the series itself.  The
 *   coefficient layout is unchanged (full [K_theta][K_phi] arrays; the
 *   m < 0 half is not read).
 *   opts may be NULL.  stream is a hipStream_t (NULL: the null stream).
 *   The plan owns every device workspace; it allocates on the current device.
 *   Errors: ERR_ARG, ERR_EPS_RANGE, ERR_ALLOC, ERR_HIP.  *out is set only on
 *   success.
 */
nufft2_status nufft2_plan(nufft2_prec prec, int64_t n_modes_theta, int64_t n_modes_phi,
                          int32_t n_fields, double eps, const nufft2_opts *opts,
                          void *stream, nufft2_handle *out);

/*
 * nufft2_setpts -- set the n_pts departure points (device arrays of FP64
 * longitude phi and colatitude theta, any real values: both coordinates are
 * taken modulo 2 pi on the doubled torus, so a point past a pole is given
 * as theta < 0 or theta > pi).  Wraps, splits each coordinate into a grid
 * cell and an offset in FP64, and bin-sorts the points; the result is kept
 * in the plan and reused by every exec.  The caller's arrays may be reused
 * once the plan's stream has passed this call.  n_pts = 0 is allowed.
 * Non-finite coordinates do not fail here: their outputs are NaN and
 * nufft2_check reports them.  Errors: ERR_ARG, ERR_ALLOC, ERR_HIP.
 */
nufft2_status nufft2_setpts(nufft2_handle p, int64_t n_pts, const double *phi_dev,
                            const double *theta_dev);

/*
 * nufft2_setpts_vector -- nufft2_setpts for a plan whose fields include the
 * east and north components (u, v) of a vector field: fields field_u and
 * field_v.  Every following nufft2_exec returns them in the frame of each
 * point's arrival point, p u + q v and -q u + p v (section 3: the matrix
 * Q = [[p, q], [-q, p]], p and q as printed after eq. sslforceb), applied
 * inside the gather before the values are stored; the other fields are as
 * with nufft2_setpts.
 *   phi_a_dev, theta_a_dev  FP64 arrival longitude / colatitude of each
 *               point (device, n_pts each, the caller's point order), read
 *               during this call only.
 *   p and q are computed here, once per point: in FP64 for FP64 plans; for
 *   FP32 plans the angles are reduced in FP64 and the sines and cosines
 *   taken in FP32 (about 1e-7 relative).  Undefined for antipodal pairs.
 *   Applies to both parts of complex outputs.  The plan keeps one (p, q)
 *   pair per point (2 x 4 or 2 x 8 bytes).  A later nufft2_setpts (or a
 *   group setpts) drops the rotation.
 *   Errors: ERR_ARG (null pointers with n_pts > 0, fields equal or out of
 *   range, or in different gather passes: field / fields_per_pass of
 *   nufft2_info must agree), ERR_ALLOC, ERR_HIP.
 */
nufft2_status nufft2_setpts_vector(nufft2_handle p, int64_t n_pts, const double *phi_dev,
                                   const double *theta_dev, const double *phi_a_dev,
                                   const double *theta_a_dev, int32_t field_u, int32_t field_v);

/*
 * nufft2_exec -- evaluate all fields at the current points.
 *   coeffs_dev  [n_fields][n_modes_theta][n_modes_phi] complex (re, im
 *               interleaved) in the plan's precision, row-major, centred;
 *               with opts.m_major = 1, [n_fields][n_modes_phi][n_modes_theta]
 *               (entry [f][b][a] is mode n = a - n_modes_theta/2, m =
 *               b - n_modes_phi/2), the layout nufft2_analysis writes when
 *               asked (nufft2_analysis_set_layout): the theta pass then reads
 *               each mode column as one contiguous run.
 *   out_dev     [n_fields][n_pts] complex in the plan's precision, in the
 *               caller's point order; with real_output or hermitian,
 *               [n_fields][n_pts] real.
 * Both are device memory owned by the caller; they must not overlap.
 * Errors: ERR_ARG, ERR_NO_POINTS, ERR_HIP.
 */
nufft2_status nufft2_exec(nufft2_handle p, const void *coeffs_dev, void *out_dev);

/*
 * nufft2_rotate_uv -- express an interpolated vector field in the arrival
 * points' frame (section 3: the matrix Q = [[p, q], [-q, p]] applied to
 * the departure-point value, with p, q as printed after eq. sslforceb).
 *   out_dev     the output of the last nufft2_exec ([n_fields][n_pts],
 *               caller's point order); fields field_u and field_v hold the
 *               east and north components (u, v) at the departure points
 *               and are overwritten, in place, by p u + q v and -q u + p v.
 *   phi_a_dev, theta_a_dev  FP64 arrival longitude / colatitude per point;
 *   phi_d_dev, theta_d_dev  FP64 departure points (those given to setpts).
 * p and q are computed in FP64; undefined for antipodal pairs.  Applies to
 * both parts of complex outputs.  Errors: ERR_ARG (fields equal or out of
 * range, null pointers), ERR_NO_POINTS, ERR_HIP.
 */
nufft2_status nufft2_rotate_uv(nufft2_handle p, void *out_dev, int32_t field_u, int32_t field_v,
                               const double *phi_a_dev, const double *theta_a_dev, const double *phi_d_dev,
                               const double *theta_d_dev);

/*
 * nufft2_exec_noalloc -- nufft2_setpts followed by nufft2_exec in one call,
 * without a plan and without allocating device memory: for callers that
 * cannot allocate (tight serving loops, harnesses that forbid allocation).
 * It is not meant for HIP graph capture (it clears its counters with
 * memset operations and may copy tables from the host).
 *   The arguments are those of nufft2_plan (stream: a hipStream_t), of
 *   nufft2_setpts (n_pts FP64 points phi_dev, theta_dev) and of
 *   nufft2_exec (coeffs_dev, out_dev), with the same layouts; the result is
 *   the same as that sequence's on a plan of the same parameters (the same
 *   kernels run).  n_pts = 0 returns at once.
 *   Every workspace of the evaluation (tables, sorted points, bins,
 *   theta-pass output, fine grid) lives in one static device array of
 *   nufft2_noalloc_capacity() bytes (128 MiB) per GPU, held from the first
 *   call on that GPU until the process ends; an evaluation that does not
 *   fit returns ERR_ARG before anything is enqueued (the grid and theta-pass
 *   output take F nf^2 and F nf K complex values: 256 x 512 grids with three
 *   fields fit in both precisions, 1024 x 2048 grids do not).
 *   Every call on one GPU shares that array and finds the previous call's
 *   contents there: calls that overlap on one GPU (other threads, or other
 *   streams whose work is still running) race and give wrong results.  The
 *   tables (deconvolution factors, twiddles) are computed on the host and
 *   copied only when they differ from the previous call's on that GPU
 *   (the call then waits for `stream`); otherwise the call only enqueues
 *   work.  Non-finite coordinates give NaN outputs (there is no flag to
 *   check without a plan).  Errors: as nufft2_plan, nufft2_setpts and
 *   nufft2_exec; ERR_ARG also when the evaluation does not fit.
 * nufft2_noalloc_capacity -- *bytes = the size of that array.
 */
nufft2_status nufft2_exec_noalloc(nufft2_prec prec, int64_t n_modes_theta, int64_t n_modes_phi, int32_t n_fields,
                                  double eps, const nufft2_opts *opts, int64_t n_pts, const double *phi_dev,
                                  const double *theta_dev, const void *coeffs_dev, void *out_dev, void *stream);
nufft2_status nufft2_noalloc_capacity(uint64_t *bytes);

/* nufft2_destroy -- synchronise the plan's stream and free everything. NULL is ignored. */
nufft2_status nufft2_destroy(nufft2_handle p);

/* nufft2_strerror -- static text for a status. */
const char *nufft2_strerror(nufft2_status s);

/* nufft2_get_info -- copy the plan's parameters into *info (host). */
nufft2_status nufft2_get_info(nufft2_handle p, nufft2_info *info);

/*
 * nufft2_check -- synchronise the plan's stream and report device-side
 * conditions: ERR_NONFINITE if the current points hold a NaN or Inf
 * coordinate, ERR_HIP if a launch failed, else OK.
 */
nufft2_status nufft2_check(nufft2_handle p);

/* nufft2_set_stream -- move the plan to another hipStream_t (orders after the old one). */
nufft2_status nufft2_set_stream(nufft2_handle p, void *stream);

/*
 * Stage timing with HIP events on the plan's stream.
 *   stage 0  setpts (wrap/split, bin count, scan, scatter)
 *         1  theta pass (deconvolution, padding, FFT over n)
 *         2  phi pass (FFT over m of the reached rows)
 *         3  gather (kernel interpolation at the points)
 * nufft2_profile_enable -- from now on bracket the stages whose bit is set in
 *   stage_mask with a pair of events (0 stops).  Events cost a few
 *   microseconds of queue time each; leave profiling off when not measuring.
 * nufft2_profile_read -- synchronise the stream, add up the elapsed time of
 *   every bracketed launch since the last read into total_ms[4] (host array,
 *   milliseconds) and their number into count[4], and reset.
 */
#define NUFFT2_N_STAGES 4
nufft2_status nufft2_profile_enable(nufft2_handle p, uint32_t stage_mask);
nufft2_status nufft2_profile_read(nufft2_handle p, double *total_ms, int64_t *count);

/*
 * Groups: many plans run as one unit, for ensembles whose members have
 * uneven grid sizes (section 5's evaluation repeated for every member and
 * field).  Members whose plans share precision, mode counts, field count,
 * kernel width and shape, tiles and output kind form a class; a group runs
 * each setpts kernel once per precision over all members' points, and each
 * exec stage once per class over all of the class's members, as
 * segmented launches captured in one HIP graph per call type; in the exec
 * graph the classes are parallel branches (up to 4, on side streams the
 * group owns), so one class's kernels overlap another's.  Results are
 * bit-identical to running every plan on its own.
 *
 * nufft2_group_create -- group the n distinct plans (host array of handles).
 *   All plans must use the same stream and device; the group keeps pointers
 *   to them, and they must outlive the group.  The group owns a stream of
 *   its own (ordered after and before the plans' stream with events, so
 *   calls keep the plans' stream order), up to three side streams for the
 *   exec branches (default priority) and small device tables.
 *   Errors: ERR_ARG (n < 1, null or repeated plan, mixed streams or
 *   devices), ERR_ALLOC, ERR_HIP.
 * nufft2_group_setpts -- nufft2_setpts for every member: n_pts[i] points at
 *   phi_dev[i], theta_dev[i] (host arrays of n entries).  Same argument
 *   rules and device-side behaviour as nufft2_setpts.
 * nufft2_group_exec -- nufft2_exec for every member: coeffs_dev[i],
 *   out_dev[i] (host arrays of n device pointers, none null, also for
 *   members with zero points).  Errors: ERR_ARG, ERR_NO_POINTS (a member
 *   without points set), ERR_HIP.
 *   A change of any device pointer or point count since the previous call
 *   of the same kind rewrites the group's tables (it first waits for the
 *   group's earlier work); a change of the total point count also
 *   re-captures the setpts graph.
 * nufft2_group_run -- nufft2_group_setpts then nufft2_group_exec as one
 *   graph launch (every setpts and exec kernel of the group in one HIP
 *   graph, captured on first use and again when the setpts launches change
 *   shape), from one host call: the GPU does not wait for the host between
 *   the two.  Arguments and errors as the two calls; on an error nothing is
 *   launched and the members keep their previous points.
 * nufft2_group_destroy -- synchronise and free the group (not the plans).
 * nufft2_group_get_info -- members, classes and the kernels per graph.
 */
typedef struct nufft2_group_s *nufft2_group;
typedef struct {
    int32_t n_members;
    int32_t n_classes;          /* exec classes */
    int32_t setpts_kernels;     /* kernels in the setpts graph */
    int32_t exec_kernels;       /* kernels in the exec graph */
    uint64_t table_bytes;       /* device memory of the group's tables */
} nufft2_group_info;

nufft2_status nufft2_group_create(const nufft2_handle *plans, int32_t n, nufft2_group *out);
nufft2_status nufft2_group_setpts(nufft2_group g, const int64_t *n_pts, const double *const *phi_dev,
                                  const double *const *theta_dev);
nufft2_status nufft2_group_exec(nufft2_group g, const void *const *coeffs_dev, void *const *out_dev);
nufft2_status nufft2_group_run(nufft2_group g, const int64_t *n_pts, const double *const *phi_dev,
                               const double *const *theta_dev, const void *const *coeffs_dev, void *const *out_dev);
nufft2_status nufft2_group_destroy(nufft2_group g);
nufft2_status nufft2_group_get_info(nufft2_group g, nufft2_group_info *info);

/*
 * nufft2_autotune -- choose the kernel width and gather tiles for a problem
 * (the same shape, tolerance and point distribution as the caller's).
 *   Width: the rule w0 = ceil(log10(1/eps)) + 1 is a guide, not the answer:
 *   for w = w0 - 1, w0, ... below the reference width min(16, w0 + 3) the
 *   tuner measures the relative l2 error of a plan of width w against an
 *   FP64 plan of the reference width on the first min(n_pts, 16384) of the
 *   caller's points and one field of pseudo-random coefficients with a flat
 *   spectrum (the hardest case for a given tolerance), and keeps the
 *   smallest w whose error is <= eps.  If none is (eps at the precision's
 *   floor), it returns ERR_EPS_RANGE with result->w and result->err of the
 *   widest candidate, and writes nothing to the cache.
 *   Tiles: for that width it times setpts + exec of n_fields fields on all
 *   n_pts points (HIP events on `stream`, median of 3 after a warm-up) for
 *   each gather tile shape in a fixed candidate list that fits the LDS, and
 *   keeps the fastest.
 *   cache_path (may be NULL): a JSON file of earlier results, keyed by
 *   precision, mode counts, fields, eps, point count rounded up to a power of
 *   two and the device's architecture name; a hit skips the measurements,
 *   a miss adds an entry (the file is rewritten through a temporary file).
 *   opts_out: on input, hermitian = 1 times the tiles on real-field plans
 *   (odd mode counts; the width search is the same), 0 on complex ones (its
 *   other input fields are ignored); on output it receives w, tile_theta,
 *   tile_phi and hermitian (other fields zero), ready for nufft2_plan;
 *   result (may be NULL) the measured error, time and whether the cache
 *   answered.  The tuner creates and destroys its own plans and buffers on
 *   the current device and synchronises `stream`.
 *   Errors: as nufft2_plan for the arguments (n_pts must be >= 1),
 *   ERR_EPS_RANGE (no width reaches eps, see above), ERR_ALLOC, ERR_HIP.
 */
typedef struct {
    int32_t w, tile_theta, tile_phi;
    int32_t from_cache;   /* 1: read from the cache file */
    double err;           /* relative l2 error of the chosen width on the probe */
    double ms;            /* setpts + exec time of the chosen configuration */
    int32_t n_timed;      /* configurations timed */
    int32_t reserved;
} nufft2_tune_result;

nufft2_status nufft2_autotune(nufft2_prec prec, int64_t n_modes_theta, int64_t n_modes_phi, int32_t n_fields,
                              double eps, int64_t n_pts, const double *phi_dev, const double *theta_dev,
                              void *stream, const char *cache_path, nufft2_opts *opts_out,
                              nufft2_tune_result *result);

/*
 * nufft2_autotune_group -- nufft2_autotune for plans that will run as
 * members of a group (nufft2_group_*).  The width is chosen as above; each
 * tile candidate is timed as a group of `members` plans of that shape, every
 * member with the caller's n_pts points (group setpts + group exec), so the
 * tiles are judged at the occupancy the ensemble runs at rather than at one
 * member's.  members: 1 .. 4096, members * n_pts < 2^31 (else ERR_ARG);
 * members = 1 is nufft2_autotune.  The cache key records members.  The tuner
 * allocates members outputs of n_fields * n_pts values besides the plans.
 */
nufft2_status nufft2_autotune_group(nufft2_prec prec, int64_t n_modes_theta, int64_t n_modes_phi, int32_t n_fields,
                                    double eps, int32_t members, int64_t n_pts, const double *phi_dev,
                                    const double *theta_dev, void *stream, const char *cache_path,
                                    nufft2_opts *opts_out, nufft2_tune_result *result);

/*
 * Serving: a request loop that evaluates independent interpolation requests
 * of mixed size and tolerance (section 5's evaluation, one request per
 * point set) with continuous batching.  A scheduler thread admits queued
 * requests in arrival order as soon as an in-flight slot is free and the
 * request's device footprint (its plan's workspaces and its own input and
 * output buffers) fits the HBM budget; admitted requests run on their
 * slot's stream, so requests that arrive while others are on the GPU
 * overlap with them.  Plans are cached by (precision, modes, fields, eps)
 * and reused; idle cached plans are destroyed, least recently used first,
 * when their memory is needed.  A request's result does not depend on what
 * else runs with it (each runs on its own plan and buffers).
 *
 * nufft2_server_create -- opts: hbm_budget bytes of device memory for plans
 *   and request buffers (0: 16 GiB), max_inflight requests on the device at
 *   once (0: 8, at most 64).  The server owns one stream per slot (default
 *   priority), a pinned host staging buffer per slot for discarded outputs,
 *   and the scheduler thread; it runs on the current device.
 *   Errors: ERR_ARG, ERR_ALLOC, ERR_HIP.
 * nufft2_server_submit -- queue one request (returns at once).  The host
 *   buffers must stay valid and unchanged until the request completes;
 *   pinned memory lets the copies overlap with other work.  out_host may be
 *   NULL: the result is copied to a server staging buffer and dropped (the
 *   copy still counts toward the latency).  t_arrival is the request's
 *   arrival time on the server clock (nufft2_server_clock); latency runs
 *   from it to the end of the device-to-host copy.  *ticket identifies the
 *   request.  Errors: ERR_ARG (bad sizes, eps, null inputs, or a request
 *   whose footprint alone exceeds the budget), ERR_EPS_RANGE.
 * nufft2_server_wait -- block until the request has completed; its status
 *   (a plan or HIP error of that request) and latency in seconds.
 * nufft2_server_stats -- counters and latency percentiles of the requests
 *   completed so far, the breakdown of their time (queue wait, copies,
 *   kernels) and the high-water mark of reserved device memory (cached
 *   plans count with their own workspace size, including point workspaces
 *   grown for larger requests, which are reserved before they are grown).
 * nufft2_server_drain -- block until every submitted request has completed.
 * nufft2_server_destroy -- drain, stop the thread, free everything.
 */
typedef struct nufft2_server_s *nufft2_server;
typedef struct {
    uint64_t hbm_budget;
    int32_t max_inflight;
    int32_t reserved;
} nufft2_server_opts;

typedef struct {
    int32_t prec;                /* nufft2_prec */
    int32_t n_fields;
    int64_t n_modes_theta, n_modes_phi;
    double eps;
    int64_t n_pts;               /* >= 1 */
    const void *coeffs_host;     /* [n_fields][Kt][Kp] complex, plan precision */
    const double *phi_host, *theta_host;  /* [n_pts] each */
    void *out_host;              /* [n_fields][n_pts] complex, or NULL */
    double t_arrival;            /* seconds, server clock */
} nufft2_request;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t points_fields;       /* sum over completed requests */
    double latency_p50, latency_p99, latency_max;  /* seconds */
    double first_arrival, last_completion;          /* server clock */
    int64_t plans_created, plans_evicted;
    uint64_t hbm_high_water;     /* bytes reserved at most at once */
    int32_t max_inflight_seen;
    int32_t reserved;
    /* where a completed request's time went (seconds, p50 and p99 over the
     * completed requests): queue wait from arrival to admission, the
     * host-to-device copies, setpts + exec, the device-to-host copy (the
     * last three from HIP events on the request's stream) */
    double queue_p50, queue_p99, h2d_p50, h2d_p99, kernel_p50, kernel_p99, d2h_p50, d2h_p99;
} nufft2_server_stats_t;

nufft2_status nufft2_server_create(const nufft2_server_opts *opts, nufft2_server *out);
double nufft2_server_clock(nufft2_server s);
nufft2_status nufft2_server_submit(nufft2_server s, const nufft2_request *req, uint64_t *ticket);
nufft2_status nufft2_server_wait(nufft2_server s, uint64_t ticket, nufft2_status *req_status, double *latency);
nufft2_status nufft2_server_drain(nufft2_server s);
nufft2_status nufft2_server_stats(nufft2_server s, nufft2_server_stats_t *stats);
nufft2_status nufft2_server_destroy(nufft2_server s);

/*
 * DFS analysis (section 4): fields sampled on Grid [0] -> the exp-form
 * coefficients nufft2_exec takes, so callers can start from grid values.
 * Grid [0] with J latitudes: row i is colatitude theta_i = (i + 1/2) pi / J
 * (i < J), column k longitude phi_k = pi k / J (k < 2J).  The paper
 * computes the standard-DFS coefficients with an FFT in phi and cosine (even
 * m) / sine (odd m) transforms in theta, and maps them to exp form with
 * eq. dfs_fourier_coeffs; the library computes the same coefficients as one
 * forward transform per phi mode over the theta circle doubled by the glide
 * reflection (which is the even / odd extension of those transforms), with
 * the half-cell theta phase.  Truncation N = M = J - 1, i.e. the output is
 * [n_fields][2J-1][2J-1] complex in the plan precision, centred exactly as
 * nufft2_exec's input (row a <-> n = a - (J-1), column b <-> m = b - (J-1)).
 * Samples of a field band-limited to |n|, |m| <= J - 1 are reproduced
 * exactly (to rounding) by nufft2_exec at the nodes.
 *
 * nufft2_analysis_plan -- J a power of two, 16 <= J <= 2048; prec as for
 *   nufft2_plan; stream a hipStream_t.  Owns its tables and a
 *   [n_fields][J][2J-1] complex buffer.  Errors: ERR_ARG, ERR_ALLOC, ERR_HIP.
 * nufft2_analysis_exec -- values_dev [n_fields][J][2J] real (plan precision,
 *   row-major), coeffs_dev [n_fields][2J-1][2J-1] complex; device memory
 *   owned by the caller, not overlapping.  Asynchronous on the plan's stream.
 *   Errors: ERR_ARG, ERR_HIP.
 * nufft2_analysis_destroy -- synchronise the stream and free; NULL ignored.
 */
typedef struct nufft2_analysis_s *nufft2_analysis;
nufft2_status nufft2_analysis_plan(nufft2_prec prec, int64_t J, int32_t n_fields, void *stream,
                                   nufft2_analysis *out);
nufft2_status nufft2_analysis_exec(nufft2_analysis a, const void *values_dev, void *coeffs_dev);
nufft2_status nufft2_analysis_destroy(nufft2_analysis a);

/*
 * nufft2_analysis_set_zonal_filter -- the zonal filter of section 4 for the
 * following nufft2_analysis_exec calls: at Grid [0] colatitude theta_i the
 * longitudinal wavenumbers m > M_zf(theta_i) = min(M, M0 + M sin theta_i),
 * M = J - 1, are removed from the samples before the theta transforms (the
 * same as filtering the grid values row by row first).  The paper uses
 * M0 = 20.  M0 < 0 turns the filter off (the default).  Synchronises the
 * plan's stream.  Errors: ERR_ARG (null handle), ERR_HIP.
 */
nufft2_status nufft2_analysis_set_zonal_filter(nufft2_analysis a, int32_t M0);

/*
 * nufft2_analysis_set_layout -- the output layout of the following
 * nufft2_analysis_exec calls: m_major = 0 (the default) writes
 * [n_fields][2J-1 (n)][2J-1 (m)], m_major = 1 writes
 * [n_fields][2J-1 (m)][2J-1 (n)], the layout of a plan created with
 * opts.m_major = 1 (its theta pass then reads whole mode columns).  The
 * same values either way.  Errors: ERR_ARG.
 */
nufft2_status nufft2_analysis_set_layout(nufft2_analysis a, int32_t m_major);

/*
 * Partial-regularity DFS expansion (section 4, eq. pr_dfs).  Column m of
 * the basis multiplies cos(m phi) and sin(m phi) by
 *   m = 0: cos(n theta), n = 0..N;          m = 1: sin(theta) cos(n theta), n = 0..N-1;
 *   even m >= 2: sin(theta) sin(n theta), n = 1..N-1;
 *   odd m >= 3: sin^2(theta) sin(n theta), n = 1..N-2.
 * Layouts (device memory owned by the caller, not overlapping):
 *   coeffs  [n_fields][2N+1][2M+1] complex in the plan precision, exp form
 *           (eq. std_dfs_exp), centred exactly as nufft2_exec's input with
 *           K_theta = 2N+1, K_phi = 2M+1 (and as nufft2_analysis_exec's output
 *           with N = M = J - 1);
 *   pr      [n_fields][2][N+1][M+1] real in the plan precision: [f][0][n][m]
 *           multiplies cos(m phi), [f][1][n][m] sin(m phi); entries outside a
 *           column's range are written as zero and ignored on input.
 *
 * nufft2_pr_plan -- 5 <= N, M <= 2047, 1 <= n_fields <= 64; stream a
 *   hipStream_t.  Factors the four per-class normal matrices on the host and
 *   owns them plus an FP64 work buffer of 16 (N+1)(M+1) n_fields bytes.
 *   Errors: ERR_ARG, ERR_ALLOC, ERR_HIP.
 * nufft2_pr_project -- least-squares projection (section 4): reads coeffs as
 *   standard coefficients (the least-squares inverse of
 *   eq. dfs_fourier_coeffs, exact for real DFS fields) and writes the pr
 *   coefficients whose residual is orthogonal to every basis function of
 *   its column (the printed conditions; tridiagonal and pentadiagonal
 *   systems per column).  Computed in FP64 for both precisions.
 * nufft2_pr_synthesize -- pr coefficients -> exp-form coefficients (the
 *   conversion after eq. std_dfs, then eq. dfs_fourier_coeffs), computed in
 *   FP64 and rounded once.  For even m >= 2 the standard n = 0 coefficient
 *   is f_{1,m} / 2 (the constant term of sin(theta)^2; the printed 0 would
 *   not vanish at the poles).
 * Both are asynchronous on the plan's stream.  Errors: ERR_ARG, ERR_HIP.
 * nufft2_pr_destroy -- synchronise the stream and free; NULL ignored.
 */
typedef struct nufft2_pr_s *nufft2_pr;
nufft2_status nufft2_pr_plan(nufft2_prec prec, int64_t N, int64_t M, int32_t n_fields, void *stream,
                             nufft2_pr *out);
nufft2_status nufft2_pr_project(nufft2_pr h, const void *coeffs_dev, void *pr_dev);
nufft2_status nufft2_pr_synthesize(nufft2_pr h, const void *pr_dev, void *coeffs_dev);
nufft2_status nufft2_pr_destroy(nufft2_pr h);

/*
 * DFS coefficients from samples on the Gauss-Legendre grid (section 2,
 * eq. GLGrid; section 5, the interpolation used for the SHT model).  Row j
 * of the grid is colatitude theta_j = arccos(z_j), z_j the roots of the
 * degree-J Legendre polynomial, in increasing theta; column k is longitude
 * phi_k = pi k / J.  After an FFT in longitude (|m| <= J - 1), each m is
 * interpolated in latitude in the standard DFS parity: cos(n theta),
 * n = 0..J-1, for even m and sin(n theta), n = 1..J, for odd m, by the
 * inverses of the two J x J latitude matrices (formed once per plan from
 * their LU factors in long double; applied on the matrix cores).  The
 * output is the exp form of eq. std_dfs_exp with n = -J..J and
 * m = -(J-1)..J-1: [n_fields][2J+1][2J-1] complex in the plan precision,
 * centred (row a <-> n = a - J, column b <-> m = b - (J-1)), the input of
 * nufft2_exec with K_theta = 2J+1, K_phi = 2J-1.  The series it defines
 * takes the (longitude-truncated) samples at the grid nodes.
 *
 * nufft2_gl_nodes -- host helper: theta[J] (host array of J doubles), the
 *   grid's colatitudes.  1 <= J <= 4096.  Errors: ERR_ARG.
 * nufft2_gl_plan -- J a power of two, 16 <= J <= 1024; prec as for
 *   nufft2_plan; stream a hipStream_t.  Owns the inverses (2 J^2 reals),
 *   twiddle tables and an [n_fields][J][2J-1] complex buffer.  Plan creation
 *   inverts two J x J matrices on the host (about a second at J = 1024).
 *   Errors: ERR_ARG, ERR_ALLOC, ERR_HIP.
 * nufft2_gl_exec -- values_dev [n_fields][J][2J] real (plan precision,
 *   row-major), coeffs_dev as above; device memory owned by the caller, not
 *   overlapping.  Asynchronous on the plan's stream.  Errors: ERR_ARG, ERR_HIP.
 * nufft2_gl_destroy -- synchronise the stream and free; NULL ignored.
 */
typedef struct nufft2_gl_s *nufft2_gl;
nufft2_status nufft2_gl_nodes(int64_t J, double *theta);
nufft2_status nufft2_gl_plan(nufft2_prec prec, int64_t J, int32_t n_fields, void *stream, nufft2_gl *out);
nufft2_status nufft2_gl_exec(nufft2_gl g, const void *values_dev, void *coeffs_dev);
nufft2_status nufft2_gl_destroy(nufft2_gl g);

/*
 * Host-only helpers (no device work; usable without a GPU).
 *
 * nufft2_kernel_params -- the width and shape the plan would choose for eps
 * and prec (same rule as nufft2_plan).
 *
 * nufft2_kernel_correction -- the deconvolution factors for K centred modes
 * on an nf-point grid:  corr[a] = 2 / (w * Phi(pi * w * k / nf)),
 * k = a - K/2, with Phi(xi) = int_{-1}^{1} exp(beta (sqrt(1 - z^2) - 1)) cos(xi z) dz
 * evaluated by Gauss-Legendre quadrature in FP64.  corr is a host array of K doubles.
 */
nufft2_status nufft2_kernel_params(nufft2_prec prec, double eps, int32_t *w, double *beta);
nufft2_status nufft2_kernel_correction(int64_t K, int64_t nf, int32_t w, double beta,
                                       double *corr);

/*
 * Diagnostics for stage tests: a read-only view of a plan workspace.
 *   which 0: fine grid   [n_fields][nf_theta][nf_phi] complex, real for
 *                        real-field plans (rows not touched by the current
 *                        points are stale)
 *         1: point records in bin order (struct {int32 i0_theta, i0_phi;
 *            real v_theta, v_phi}; real = plan precision)
 *         2: permutation, int32 [n_pts]: record r belongs to point perm[r]
 *         3: bin starts, int32 [n_bins + 1] (bin b holds records
 *            start[b] .. start[b+1]-1)
 *         4: theta rows reached by the current points' taps, uint8 [nf_theta]
 *         5: theta-pass output [n_fields][nf_theta][n_modes_phi] complex
 *            (real-field plans: [n_fields][nf_theta][n_modes_phi/2 + 1],
 *            modes m = 0 .. n_modes_phi/2)
 *         6: non-empty bins, int32 [n_bins + 1]: the first k entries are the
 *            bins holding at least one record in increasing order, entry
 *            n_bins is k
 * *dev_ptr and *bytes describe device memory the plan owns; valid until the
 * next setpts or destroy.  Errors: ERR_ARG, ERR_NO_POINTS (points-derived
 * buffers before setpts).
 */
nufft2_status nufft2_debug_buffer(nufft2_handle p, int32_t which, void **dev_ptr,
                                  uint64_t *bytes);

#ifdef __cplusplus
}
#endif

#endif /* NUFFT2_H */
