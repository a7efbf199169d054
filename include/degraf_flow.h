/*
 * degraf_flow.h -- C ABI of the MI355X (gfx950) DeGraF key-point detector and robust local
 * optical flow tracker.
 *
 * Method: Stephenson, Breckon, Katramados, "DeGraF-Flow: Extending DeGraF Features for accurate
 * and efficient sparse-to-dense optical flow estimation" (2019), Section 2: points are detected
 * on a uniform grid of gradient centroids in the first frame ("Point detection", Eq. 1-2 and the
 * selection rule) and tracked into the next frame with robust local optical flow ("Sparse point
 * tracking"; the RLOF(IM-GM) options of Section 3 "Parameters" as flags), and the tracked points
 * can be interpolated into a dense field ("Interpolation", dgf_epic).
 *
 * Conventions shared by every call:
 *   - Every data pointer is a DEVICE pointer owned by the caller.  The library never allocates
 *     or frees caller memory; only a batch plan (dgf_batch_*) owns device memory, released by
 *     dgf_batch_destroy.
 *   - Every compute call is asynchronous on `stream` (a hipStream_t passed as void*, NULL = the
 *     default stream), performs no host synchronisation and no device allocation.
 *   - Return value: DGF_OK (0) or a negative DGF_ERR_* code.  Arguments are validated on the host
 *     before anything is launched; on error nothing is launched and outputs are untouched.
 *     Numerical trouble on the device (flat texture, divergence, non-finite pixels) is reported
 *     per point through `status`, never as an error code.
 *   - Coordinates: x = column, y = row, pixel centres at integer coordinates.  Points are float
 *     pairs (x, y); flow[k] is the displacement u with I1(p_k + u) ~ I0(p_k).
 *   - Images are row-major with a row pitch in bytes (pitch >= width * element size).
 */
#ifndef DEGRAF_FLOW_H
#define DEGRAF_FLOW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------------------------- */
#define DGF_OK 0
#define DGF_ERR_INVALID_ARG (-1) /* null pointer, bad size, bad dtype, bad pitch, ...          */
#define DGF_ERR_CAPACITY (-2)    /* output capacity smaller than the number of results          */
#define DGF_ERR_UNSUPPORTED (-3) /* valid request outside what the library implements         */
#define DGF_ERR_HIP (-4)         /* a HIP runtime call or kernel launch failed                   */
#define DGF_ERR_WORKSPACE (-5)   /* workspace null or smaller than dgf_track_workspace_bytes()   */
#define DGF_ERR_SCRATCH (-6)     /* input larger than the static scratch of dgf_track_static     */

/* ---- per-point tracking status ----------------------------------------------------------------- */
#define DGF_ST_CONVERGED 0       /* level 0 stopped on the step-size test, p + u inside image    */
#define DGF_ST_NOT_CONVERGED 1   /* level 0 ran out of iterations, or a step was not finite     */
#define DGF_ST_ILL_CONDITIONED 2 /* lambda_min(G0) / s^2 < min_eig at level 0 (u = the guess) */
#define DGF_ST_OUT_OF_BOUNDS 3   /* input point, or converged p + u, outside [0,W-1] x [0,H-1]  */

/* ---- element types ------------------------------------------------------------------------------ */
#define DGF_U8 0  /* uint8 grey levels 0..255 */
#define DGF_F32 1 /* float, same 0..255 scale for the default tracker constants */

#define DGF_MAX_LEVELS 12
#define DGF_MAX_WINDOW 128
#define DGF_MAX_SUPPORT 31

typedef struct {
    const void *data;    /* device pointer to row 0                                   */
    int32_t width;       /* columns, >= 1                                             */
    int32_t height;      /* rows, >= 1                                                */
    int64_t pitch_bytes; /* bytes between consecutive rows, >= width * element size;
                            pitch_bytes < 2^24, height < 2^24 and pitch_bytes * height
                            < 2^31 (2 GiB); larger images are rejected                 */
    int32_t dtype;       /* DGF_U8 or DGF_F32                                         */
} dgf_image;

/* Robust tracker constants.  The paper leaves the tracker's norm and stopping rule to its
 * citation; this library uses a continuous, piecewise-linear redescending influence function
 *   psi(r) = r (|r| <= sigma1),  sign(r) sigma1 (sigma2 - |r|) / (sigma2 - sigma1)
 *            (sigma1 < |r| < sigma2),  0 (|r| >= sigma2)
 * with iteratively re-weighted Gauss-Newton steps, w = psi(r) / r. */
typedef struct {
    float sigma1;     /* inner threshold, intensity units (default 8)                   */
    float sigma2;     /* outer threshold, intensity units (default 32); both INFINITY
                         gives plain least-squares pyramidal Lucas-Kanade; sigma1 >=
                         sigma2 gives a hard cutoff at sigma1; a finite sigma1 with an
                         infinite sigma2 is rejected (DGF_ERR_INVALID_ARG)               */
    float eps_coarse; /* a level > 0 stops when |step|_2 < eps_coarse px (default 1e-2) */
    float eps_fine;   /* level 0 stops when |step|_2 < eps_fine px (default 1e-4)       */
    float min_eig;    /* a level with lambda_min(G0)/|support| < min_eig runs no iteration
                         and passes its guess on; at level 0 the point is ill-conditioned
                         (default 1e-4 * 255^2); |support| = s^2 for the square window  */
    int32_t flags;    /* 0, or any of DGF_TRACK_ILLUM, DGF_TRACK_CROSS, DGF_TRACK_GLOBAL  */
    float cross_tau;  /* DGF_TRACK_CROSS: arm threshold, intensity units (default 25)   */
} dgf_track_opts;

/* dgf_track_opts.flags: match each support under a per-point gain and offset estimated with
 * the flow, I1(p + k + u) ~ (1 + m) I0(p + k) + c (the illumination model of the tracker the
 * paper runs, RLOF(IM), Section 3 "Parameters"; the model itself is defined in its citation).
 * Each iteration then solves a 4x4 system in (d, m, c), with residual derivatives
 * ((1 + m) g, -T, -1); m and c start at 0 and carry over between levels; a point whose final
 * gain 1 + m lies outside [1/2, 2] is NOT_CONVERGED (a contrast change, not a match).  Supported for the
 * supports the row-run kernel is compiled for (5, 7, 9, 11, 15, 21), else DGF_ERR_UNSUPPORTED.
 * dgf_track_backward and dgf_batch_backward differentiate it given the forward call's
 * (gain, offset) (illum_out). */
#define DGF_TRACK_ILLUM 1

/* dgf_track_opts.flags: adaptive cross-based supports (the support region RLOF(IM-GM) uses,
 * Section 3 "Parameters"; defined in its citation).  At every level the region is decided on the
 * level image's own pixels at floor(p_l) + k, k in [-r-1, r+1]^2 (border replicated): the vertical
 * arm of the centre runs up and down while each next centre-column pixel stays within cross_tau
 * of the centre, every row it covers gets a horizontal arm around its centre-column pixel (within
 * cross_tau of that pixel), and the support keeps the window offsets that lie, with their four
 * neighbours (the stencil of the template gradient), in the union of those arms.  Every support sum runs over the kept pixels
 * and the trackability test divides by their number.  Supports of the row-run kernel only
 * (5, 7, 9, 11, 15, 21; else DGF_ERR_UNSUPPORTED); not differentiated (dgf_track_backward and
 * dgf_batch_backward reject it). */
#define DGF_TRACK_CROSS 2

/* dgf_track_opts.flags: global-motion prior (the "GM" of RLOF(IM-GM), Section 3 "Parameters";
 * defined in its citation).  A first pass tracks every point on the coarsest level alone from zero
 * motion; the points that stop there on the step test give samples (their motion at their
 * level-0 position) of one global affine motion v = A (x - (W-1)/2, y - (H-1)/2, 1)^T, fitted by
 * least squares and then ten Tukey-biweight reweightings (scale 4.685 coarsest-level pixels);
 * with fewer than 3 samples or collinear positions the model is their weighted mean motion, with
 * none it is zero.  The tracking proper then starts each point on the coarsest level from
 * A p~ / 2^(levels-1) instead of zero.  All of it runs on the stream (no host synchronisation);
 * the model lives in the workspace (dgf_track_workspace_bytes covers it, also for levels = 1).
 * Row-run supports only, as DGF_TRACK_CROSS.  After the call the fitted model (6 doubles, A
 * row-major) sits at byte offset 2 * dgf_pyramid_layout(width, height, levels, dtype) of the
 * workspace (batch plans keep theirs inside the plan).  The gradient at a converged point does not
 * depend on where the iteration started, so the adjoint accepts the flag. */
#define DGF_TRACK_GLOBAL 4

/* Workspace bytes of dgf_gm_fit (a constant: the fit keeps at most 256 partial-sum slots). */
size_t dgf_gm_workspace_bytes(void);

/* Global affine motion of one frame from tracked points: the fit of the DGF_TRACK_GLOBAL prior
 * (Section 3 "Parameters", the "GM" of RLOF(IM-GM); defined in its citation), on any tracking result.
 * Samples are the points with status DGF_ST_CONVERGED and finite flow; v = A p~ with
 * p~ = (x - (width-1)/2, y - (height-1)/2, 1), fitted by least squares and then ten Tukey-biweight
 * reweightings, w = (1 - (e / c)^2)^2 for a residual norm e < c = 4.685 scale, else 0.  With fewer
 * than 3 weighted samples, or weighted positions whose covariance C has det C <= 1e-4 (tr C)^2, a
 * pass's model is the weighted mean motion; a pass with no weighted sample (or a singular system)
 * keeps the model before it, and with no sample at all A = 0.  FP64 throughout.
 *   points, flow  device, [n][2] float (flow in the same pixels as the points)
 *   status        device, [n]
 *   scale         > 0, finite: the Tukey scale in pixels (the tracker uses 2^(levels-1))
 *   workspace     device, >= dgf_gm_workspace_bytes() bytes
 *   model         device, 6 doubles: A row-major (2 x 3), written on `stream`
 * Errors: DGF_ERR_INVALID_ARG, DGF_ERR_WORKSPACE, DGF_ERR_HIP.  Nothing is launched on an error. */
int dgf_gm_fit(const float *points, const float *flow, const uint8_t *status, int64_t n, int32_t width,
               int32_t height, double scale, void *workspace, size_t ws_bytes, double *model, void *stream);

/* ---- library ----------------------------------------------------------------------------------- */

/* Static, NUL-terminated description of an error code (never NULL). */
const char *dgf_strerror(int code);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int dgf_version(void);

/* Fills *out with the default tracker constants listed in dgf_track_opts.  Returns DGF_OK, or
 * DGF_ERR_INVALID_ARG for a null pointer. */
int dgf_track_opts_default(dgf_track_opts *out);

/* ---- DeGraF detection (Section 2 "Point detection", Eq. 1-2 and the selection rule) --------- */

/* Number of key-points for a W x H image: one per window position, windows fully inside the
 * image at origins (kx * stride, ky * stride):
 *   N = (floor((W - window) / stride) + 1) * (floor((H - window) / stride) + 1), 0 if the image
 * is smaller than the window.  Pure host function; returns -1 for window/stride < 1. */
int64_t dgf_detect_count(int32_t width, int32_t height, int32_t window, int32_t stride);

/* One key-point per window (square window x window), in row-major window order: point n belongs
 * to window (n % nx, n / nx).  For each window the positive centroid (intensity-weighted mean
 * position, Eq. 1) and the negative centroid (weights 1 + m - I with m the window maximum, Eq. 2)
 * are formed; the key-point is the negative one when its weight sum is strictly larger, else the
 * positive one.  Sums are exact integers; the final divisions are IEEE single precision.
 *   I0       : DGF_U8 image (device)
 *   window   : 1 .. DGF_MAX_WINDOW;  stride >= 1
 *   points   : out, float[capacity][2] (x, y) in image pixels
 *   sel      : out, nullable, uint8[capacity]: 1 when the negative centroid was kept
 *   response : out, nullable, float[capacity]: |C_pos - C_neg| (C_pos := window centre for an
 *              all-zero window)
 *   capacity : number of points the outputs can hold; DGF_ERR_CAPACITY if smaller than
 *              dgf_detect_count(...).  N = 0 launches nothing and returns DGF_OK. */
int dgf_detect(const dgf_image *I0, int32_t window, int32_t stride, float *points, uint8_t *sel,
               float *response, int64_t capacity, void *stream);

/* ---- image pyramid (coarse-to-fine tracking) --------------------------------------------------- */

/* Level l+1 is the 5-tap binomial [1 4 6 4 1]/16 smoothing of level l in both directions with
 * replicated borders, sampled at even pixels: size ceil(W_l/2) x ceil(H_l/2), so a level-0
 * point p sits at p / 2^l.  uint8 levels round half up exactly ((sum + 128) >> 8); float levels
 * divide by 256.  Level 0 is the input image itself and is not copied.
 *
 * Layout of levels 1 .. levels-1 in `dst` (also used inside the track workspace): level l
 * starts at byte offsets[l] and has row pitch pitches[l] bytes (offsets[0] = pitches[0] = 0).
 * Returns the total number of bytes, or 0 for invalid arguments.  offsets/pitches nullable. */
size_t dgf_pyramid_layout(int32_t width, int32_t height, int32_t levels, int32_t dtype,
                          int64_t *offsets, int64_t *pitches);

/* Builds levels 1 .. levels-1 of `src` into `dst` (device, dst_bytes >= dgf_pyramid_layout()). */
int dgf_pyramid(const dgf_image *src, int32_t levels, void *dst, size_t dst_bytes, void *stream);

/* ---- robust local optical flow tracking (Section 2 "Sparse point tracking") ------------------- */

/* Workspace bytes needed by dgf_track for a pair of width x height images (both pyramids). */
size_t dgf_track_workspace_bytes(int32_t width, int32_t height, int32_t levels, int32_t dtype);

/* Tracks n points from I0 to I1 (same size and dtype).  For each point, coarse to fine over
 * `levels` pyramid levels with a square support of `support` x `support` pixels (odd, 1 ..
 * DGF_MAX_SUPPORT) centred on the point:
 *   template T_k = bilinear(I0_l, p/2^l + k) and its gradient g_k (central differences,
 *   bilinearly sampled); per iteration r_k = bilinear(I1_l, p/2^l + k + guess + d) - T_k,
 *   w_k = psi(r_k)/r_k, step = (sum w g g^T)^-1 (-sum w r g)  (least-squares step if the
 *   weighted matrix is near singular), at most `iters` iterations per level; the level's result
 *   seeds the next finer level as 2 (guess + d).
 *   points    : float[n][2] level-0 coordinates (device)
 *   workspace : device, >= dgf_track_workspace_bytes(width, height, levels, dtype) bytes
 *   flow      : out, float[n][2];   status : out, uint8[n] (DGF_ST_*)
 *   iters_out : out, nullable, int32[n]: iterations run by the point summed over levels
 *   illum_out : out, nullable, float[n][2]: the level-0 gain m and offset c of the illumination
 *               model (I1(p+k+u) ~ (1+m) I0(p+k) + c, offsets in grey levels of the images);
 *               only with DGF_TRACK_ILLUM in opts->flags, else DGF_ERR_INVALID_ARG
 *   opts      : nullable (defaults)
 * n = 0 launches nothing. */
int dgf_track(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
              int32_t support, int32_t iters, const dgf_track_opts *opts, void *workspace,
              size_t ws_bytes, float *flow, uint8_t *status, int32_t *iters_out, float *illum_out,
              void *stream);

/* dgf_track without a workspace argument, for callers that cannot allocate device memory (code
 * under stream capture into a graph, allocation-free serving loops, harnesses that forbid
 * hipMalloc).  Both pyramids are built into a file-scope device array of
 * DGF_TRACK_STATIC_MAX_BYTES bytes (16 MiB) that every GPU using this library holds until the
 * process ends; the call itself allocates nothing.  Arguments, outputs and results are those of
 * dgf_track (same kernels, same launch shape), minus workspace / ws_bytes.
 *   Limit : dgf_track_workspace_bytes(width, height, levels, dtype) must not exceed
 *           DGF_TRACK_STATIC_MAX_BYTES, else DGF_ERR_SCRATCH and nothing is launched (for
 *           example 1242 x 375 uint8 at 5 levels needs 0.33 MB, 2048 x 1024 float at 6 levels
 *           5.6 MB).
 *   Races : every call on one GPU uses that GPU's one array, which keeps the last call's
 *           pyramids; two calls whose work overlaps on one GPU (different streams, or host
 *           threads) race on it.  Order them on one stream or with events.
 *   Set-up: the first call on a device looks the array's device address up (hipGetSymbolAddress,
 *           with that device current); DGF_ERR_HIP if that fails.  The device is the current
 *           HIP device, which must be the one `stream` belongs to. */
#define DGF_TRACK_STATIC_MAX_BYTES (16u << 20)
int dgf_track_static(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                     int32_t support, int32_t iters, const dgf_track_opts *opts, float *flow, uint8_t *status,
                     int32_t *iters_out, float *illum_out, void *stream);

/* ---- gradient of the tracked flow (implicit differentiation at the converged fixed point) ---- */

/* Adds dL/dI0 and dL/dI1 for an upstream gradient dflow = dL/dflow of a previous dgf_track call
 * on the same images, points and support.  At a CONVERGED point the level-0 flow u solves
 * F(u) = sum_k psi(r_k) g_k = 0; with J = dF/du = sum_k psi'(r_k) g_k grad I1(p+k+u)^T and
 * J^T mu = dflow_k, the point contributes
 *   dI1[q] -= sum_k psi'(r_k) (mu . g_k) beta_k(q)
 *   dI0[q] += sum_k psi'(r_k) (mu . g_k) alpha_k(q) - sum_k psi(r_k) mu . dg_k/dI0[q]
 * (alpha, beta: bilinear tap weights of the template and I1 samples; g_k: central differences at
 * +-1 px of the bilinear interpolant of I0).  Where the tracker's weighted system falls back to
 * least squares at the converged flow (its rule: det of sum w_k g_k g_k^T, w = psi(r)/r, at most
 * 1e-6 of the unweighted one's, or not a number), the fixed point solves sum_k r_k g_k = 0
 * instead, and the point is differentiated with psi(r) = r, psi' = 1 (for the illumination model
 * the same test on its 4x4 systems).  Points with any other status, or a singular J, contribute
 * nothing.  Points are treated as constants (detection is not differentiated).
 *   I0, I1      : DGF_F32 images (DGF_ERR_UNSUPPORTED for DGF_U8)
 *   flow,status : outputs of dgf_track for these inputs;  dflow: float[n][2]
 *   dI0, dI1    : float images of the same size, with the row pitch of I0 and I1 respectively;
 *                 ACCUMULATED into (zero them first), with device float atomics, so the order
 *                 of additions (and the last bits) is not deterministic.
 *   opts        : the tracker constants used in the forward call (nullable = defaults).
 *   dpoints     : nullable, float[n][2]: WRITTEN with dL/dp, the gradient w.r.t. the point
 *                 positions (the template moves with the point): with
 *                 K = sum_k [-psi'(r_k) g_k grad I0(p+k)^T + psi(r_k) dg_k/dp], du/dp = -J^-1 (J + K)
 *                 and dL/dp = -dflow - K^T mu; 0 for points that contribute nothing.
 *   illum       : with DGF_TRACK_ILLUM in opts->flags: float[n][2], the (gain, offset) that
 *                 dgf_track wrote to illum_out (required when n > 0); must be null otherwise.
 *                 The adjoint is then that of the illumination model's fixed point
 *                 F(u, m, c) = sum_k psi(r_k) phi_k = 0, r_k = I1(p+k+u) - (1+m) T_k - c,
 *                 phi_k = ((1+m) g_k, -T_k, -1): a 4x4 J with J^T mu = (dflow, 0, 0), and
 *   dI1[q] -= sum_k psi'(r_k) (mu . phi_k) beta_k(q)
 *   dI0[q] += sum_k [(1+m) psi'(r_k) (mu . phi_k) + psi(r_k) mu_m] alpha_k(q)
 *             - (1+m) sum_k psi(r_k) mu_u . dg_k/dI0[q];
 *                 dpoints then uses K = sum_k [-(1+m) psi'(r_k) phi_k grad I0(p+k)^T
 *                 + psi(r_k) dphi_k/dp], dphi_k/dp = ((1+m) dg_k/dp, -grad I0(p+k)^T, 0),
 *                 and dL/dp = -dflow - K^T mu. */
int dgf_track_backward(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t support,
                       const dgf_track_opts *opts, const float *flow, const uint8_t *status, const float *dflow,
                       float *dI0, float *dI1, float *dpoints, const float *illum, void *stream);

/* Gradient through detection (Section 2 Eq. 1-2, the centroid ratios taken as functions of real
 * pixel values, evaluated at the uint8 image the points were detected on): ADDS
 *   dI0[q] += dpoints[n] . d p_n / d I0[q]
 * over every window n.  Positive centroid C = sum c I / S: dC/dI(q) = (c(q) - C) / S; negative
 * centroid with weights 1 + m - I (m = window maximum, at its first maximal pixel q* in row-major
 * order): dC/dI(q) = (-(c(q) - C) + [q = q*] sum_q' (c(q') - C)) / S_neg.
 *   I0      : the DGF_U8 frame given to dgf_detect, window / stride as there
 *   sel     : uint8[n], the selection bits dgf_detect returned;  dpoints: float[n][2] = dL/dp
 *   n       : must equal dgf_detect_count(width, height, window, stride)
 *   dI0     : float map, row pitch dI0_pitch floats (>= width); accumulated with device float
 *             atomics (windows overlap when stride < window). */
int dgf_detect_backward(const dgf_image *I0, int32_t window, int32_t stride, const uint8_t *sel,
                        const float *dpoints, int64_t n, float *dI0, int64_t dI0_pitch, void *stream);

/* ---- batched form: many pairs of uneven size and point count in one pass -------------------- */

/* One frame pair of a batch: both images DGF_U8 of the same size; DeGraF grid of this pair. */
typedef struct {
    dgf_image I0, I1;
    int32_t window, stride;
} dgf_pair_desc;

typedef struct dgf_batch dgf_batch; /* opaque plan */

/* Builds a plan for detect + pyramids + track of every pair with common levels / support /
 * iters / opts.  The images are referenced by pointer (their contents may change between runs;
 * the pointers may not).  This call is the only one that allocates device memory (one buffer
 * holding every pyramid and the descriptor tables, freed by dgf_batch_destroy) and it copies the
 * tables to the device synchronously.  DGF_ERR_UNSUPPORTED if a pair's window / stride is too
 * large for the LDS-tiled detector or the support has no kernel. */
int dgf_batch_create(const dgf_pair_desc *pairs, int32_t npairs, int32_t levels, int32_t support, int32_t iters,
                     const dgf_track_opts *opts, dgf_batch **out);

/* Total number of points of all pairs (-1 for a null plan); outputs are concatenated in pair
 * order, pair i at [offsets[i], offsets[i + 1]) (offsets: host array of npairs + 1). */
int64_t dgf_batch_num_points(const dgf_batch *b);
int dgf_batch_point_offsets(const dgf_batch *b, int64_t *offsets);

/* Runs the plan on `stream`: one launch per pyramid level for all frames, one detection launch,
 * a counter reset and one persistent tracking launch.  points: out float[N][2]; flow: out
 * float[N][2]; status: out uint8[N]; iters_out: nullable int32[N]; illum_out: nullable
 * float[N][2], the gain and offset of a plan made with DGF_TRACK_ILLUM (else must be null).
 * Results equal those of per-pair dgf_detect + dgf_track with the same tuning. */
int dgf_batch_run(dgf_batch *b, float *points, float *flow, uint8_t *status, int32_t *iters_out, float *illum_out,
                  void *stream);

/* The two halves of dgf_batch_run, for callers that time, overlap or separate them (same
 * arguments; dgf_batch_run is exactly dgf_batch_front then dgf_batch_track on one stream):
 * dgf_batch_front builds every pair's pyramids into the plan and detects every pair's points
 * (Section 2 "Point detection"); dgf_batch_track tracks the points it is given from the pyramids
 * the last front call built (Section 2 "Sparse point tracking"), and may be given other points of
 * the same count (the plan's per-pair point ranges). */
int dgf_batch_front(dgf_batch *b, float *points, void *stream);
int dgf_batch_track(dgf_batch *b, const float *points, float *flow, uint8_t *status, int32_t *iters_out,
                    float *illum_out, void *stream);

/* Where the plan keeps pyramid level `level` (0 .. levels - 1) of frame `frame` (0 = I0, 1 = I1)
 * of pair `pair`, as dgf_batch_front builds it (the tracker's pyramid, Section 2 "Sparse point
 * tracking"): device pointer, row pitch in bytes, width and height; level 0 is the caller's
 * frame.  A query only (no device work).  The memory belongs to the plan, stays valid until
 * dgf_batch_destroy and is rewritten by every front or run call.  DGF_ERR_INVALID_ARG for a null
 * plan or output, or an index out of range. */
int dgf_batch_level(const dgf_batch *b, int pair, int frame, int level, const uint8_t **data, int64_t *pitch_bytes,
                    int32_t *width, int32_t *height);

/* Captures the run sequence (with these output pointers) into a HIP graph on `stream` (a created
 * stream, not the default one); dgf_batch_replay launches it with one call.  A new capture
 * replaces the previous graph. */
int dgf_batch_capture(dgf_batch *b, float *points, float *flow, uint8_t *status, float *illum_out, void *stream);
int dgf_batch_replay(dgf_batch *b, void *stream);

/* Size, in floats, of the gradient buffer dgf_batch_backward writes: every pair's dI0 then dI1,
 * each a dense width x height float map (row pitch = width), pairs in order.  offsets
 * (nullable, npairs + 1 entries) receives the first float of each pair's dI0; its dI1 starts
 * width * height floats later.  Returns -1 for a null plan. */
int64_t dgf_batch_grad_size(const dgf_batch *b, int64_t *offsets);

/* Gradient for a whole batch in one launch (the adjoint of dgf_track_backward, per pair, over
 * every point of the plan): given the points, flow and status of a dgf_batch_run / replay and an
 * upstream gradient dflow (float[num_points][2], same order), OVERWRITES grad
 * (dgf_batch_grad_size floats, device) with dL/dI0 and dL/dI1 of every pair, taking the uint8
 * frames' values as reals.  grad is cleared by a kernel first; contributions are added with
 * device float atomics, so the last bits are not deterministic.  Points that are not CONVERGED,
 * or have a singular J, contribute nothing.  illum: for a plan made with DGF_TRACK_ILLUM, the
 * gain and offset the run wrote (required, float[N][2]); null otherwise. */
int dgf_batch_backward(dgf_batch *b, const float *points, const float *flow, const uint8_t *status, const float *dflow,
                       const float *illum, float *grad, void *stream);

/* Frees the plan and its device memory (after the work using it has completed). */
int dgf_batch_destroy(dgf_batch *b);

/* ---- launch-shape tuning ------------------------------------------------------------------- */

/* Launch shape of the tracker.  It never changes results, only speed. */
typedef struct {
    int32_t lanes_per_point; /* 16, 32 or 64 lanes of a wavefront share one point            */
    int32_t waves_per_group; /* wavefronts per workgroup: 1, 2 or 4                           */
    int32_t margin;          /* I1 tile margin in pixels (clamped to what the tile allows)    */
    int32_t kernel;          /* 0: row-run pixel layout when compiled for the support, else
                                the generic layout; 1: generic layout                        */
    float ms;                /* measured time of the winning shape (dgf_autotune), else -1  */
} dgf_tuning;

/* Shape the library uses for this request (installed entry for (support, dtype), else a
 * heuristic).  Host only. */
int dgf_get_tuning(int32_t support, int32_t levels, int32_t dtype, int64_t n, dgf_tuning *out);

/* Installs a shape for (support, dtype) for the rest of the process.  Host only;
 * DGF_ERR_UNSUPPORTED if no kernel is compiled for it.  One shape serves both the plain tracker
 * and the illumination model (DGF_TRACK_ILLUM) of that support and element type. */
int dgf_set_tuning(int32_t support, int32_t dtype, const dgf_tuning *t);

/* Times every compiled launch shape on these inputs (dgf_track arguments; the pyramids are built
 * into `workspace`, flow / status receive a valid result), installs the fastest for (support,
 * dtype) and returns it in *out (nullable).  This is a setup call: it synchronises `stream`
 * once per candidate.  cache_path (nullable) names a JSON file keyed by GPU architecture,
 * support, levels, element type, the point count rounded up to a power of two and the flags
 * (DGF_TRACK_ILLUM / CROSS / GLOBAL): a hit installs the cached shape without timing anything
 * (the pyramids, flow and status are still written, by one tracking pass with that shape); a miss
 * appends the result.  The installed shape serves both models (see dgf_set_tuning), so tuning with
 * DGF_TRACK_ILLUM also sets the plain tracker's shape for this support and element type. */
int dgf_autotune(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                 int32_t support, int32_t iters, const dgf_track_opts *opts, void *workspace, size_t ws_bytes,
                 float *flow, uint8_t *status, const char *cache_path, dgf_tuning *out, void *stream);

/* The two stages of dgf_track, for callers that time or reuse them separately:
 * dgf_track_pyramids builds levels 1 .. levels-1 of both images into `workspace` (same layout
 * and size as dgf_track uses); dgf_track_run then tracks on those pyramids without rebuilding
 * them (the workspace must hold the pyramids of exactly these I0/I1 and levels).  Arguments
 * and outputs as for dgf_track. */
int dgf_track_pyramids(const dgf_image *I0, const dgf_image *I1, int32_t levels, void *workspace, size_t ws_bytes,
                       void *stream);
int dgf_track_run(const dgf_image *I0, const dgf_image *I1, const float *points, int64_t n, int32_t levels,
                  int32_t support, int32_t iters, const dgf_track_opts *opts, const void *workspace,
                  size_t ws_bytes, float *flow, uint8_t *status, int32_t *iters_out, float *illum_out,
                  void *stream);

/* dgf_detect on I0 and dgf_track_pyramids on (I0, I1) in one launch where they fit one
 * (Section 2 "Point detection"; the pyramids serve "Point tracking"): the detection tiles run
 * beside the tiles of the first pyramid-chain launch, so the two independent, latency-bound jobs
 * overlap.  Outputs are identical to the two separate calls: points / sel / response as from
 * dgf_detect(I0, window, stride, points, sel, response, capacity), and the pyramids in
 * `workspace` as from dgf_track_pyramids(I0, I1, levels, workspace, ws_bytes), ready for
 * dgf_track_run.  With levels == 1, no points, or a detection tile larger than the chain's LDS
 * (about 24 KB: (15 stride + window) rows of that many bytes), the two calls are made one after
 * the other on `stream`.
 *   I0, I1   : DGF_U8 frames of equal size (else DGF_ERR_INVALID_ARG)
 *   window, stride, points, sel, response, capacity : as for dgf_detect
 *   levels, workspace, ws_bytes : as for dgf_track_pyramids
 * Every argument is validated before anything is launched; no host synchronisation, no
 * allocation.  The caller owns every buffer. */
int dgf_detect_pyramids(const dgf_image *I0, const dgf_image *I1, int32_t window, int32_t stride, int32_t levels,
                        void *workspace, size_t ws_bytes, float *points, uint8_t *sel, float *response,
                        int64_t capacity, void *stream);

/* ---- dense flow by edge-preserving interpolation (Section 2 "Interpolation") ---------------- */

/* Interpolation constants.  k: neighbours per pixel (Section 3 "Parameters": 128), 1 .. 256.
 * kappa: cost of one pixel step on a flat image, >= 1 (default 8).  half_dist: geodesic distance
 * over which a neighbour's weight halves, >= 1 (default 64), in the same cost units. */
typedef struct {
    int32_t k;
    int32_t kappa;
    int32_t half_dist;
} dgf_epic_opts;

/* Fills *out with the defaults above.  DGF_ERR_INVALID_ARG for a null pointer. */
int dgf_epic_opts_default(dgf_epic_opts *out);

/* Workspace bytes dgf_epic needs for a width x height frame and n points (0 for bad sizes). */
size_t dgf_epic_workspace_bytes(int32_t width, int32_t height, int64_t n);

/* Dense flow for every pixel of I0 from the tracked points: each pixel q takes the affine motion
 * fitted by weighted least squares to the k points geodesically nearest to it, nearness being a
 * path cost that rises across image edges.
 *   edge map   E(x, y) = |I0(x+1, y) - I0(x-1, y)| + |I0(x, y+1) - I0(x, y-1)| (replicated border)
 *   step cost  between 4-neighbours p, q: kappa + E(p) + E(q); distances are exact integers
 *   seeds      points with status DGF_ST_CONVERGED and a finite position and flow, at pixel
 *              (floor(x + 1/2), floor(y + 1/2)) clamped into the image; a point whose pixel is
 *              that of a lower-index seed takes no part
 *   cells      D(q) = least path cost from any seed, L(q) = lowest seed index reaching q at D(q)
 *   seed graph s, t joined when their cells touch (4-adjacency), edge length = least
 *              D(p) + step(p, q) + D(q) over touching pixel pairs
 *   neighbours of q: the k seeds t smallest in (delta(L(q), t), t), delta the seed-graph distance,
 *              L(q) itself first, only those with delta <= 64 half_dist
 *   fit        weights 2^(-delta / half_dist); model u(x, y) = A (x - sx, y - sy, 1)^T about the
 *              cell seed's position (sx, sy); fewer than 3 neighbours or a weighted position
 *              covariance C with det C <= 1e-4 (tr C)^2 give the weighted mean flow
 *   dense(q)   the model of L(q) at q; NaN everywhere if there is no seed.
 * Arguments (device pointers unless noted):
 *   I0         DGF_U8 frame the points were detected on (width * height <= INT32_MAX)
 *   points, flow : float[n][2] (level-0 positions and their tracked flow); status: uint8[n]
 *   opts       nullable (defaults)
 *   workspace  >= dgf_epic_workspace_bytes(width, height, n) bytes
 *   dense      out, float rows of dense_pitch floats (even, >= 2 width), 8-byte aligned: (u, v)
 *   labels, dist : out, nullable, int32 / uint32 [height][width]: L(q) (-1 without seeds) and
 *              D(q) (0xFFFFFFFF without seeds)
 *   nbr, nbr_dist : out, nullable together, int32 / uint32 [n][k]: each seed's neighbours and
 *              graph distances in order, unused entries -1 / 0xFFFFFFFF (all for non-seeds)
 *   model      out, nullable, float[n][6]: the row-major 2x3 A of each seed (NaN for non-seeds)
 * Unlike the other calls this one synchronises `stream`: the geodesic relaxation runs until a
 * pass changes nothing, which the host reads back (dgf_epic_async below does not).  Errors: DGF_ERR_UNSUPPORTED when
 * (width + height - 2) (kappa + 1020) exceeds 2^32 - 2 (distances are 32-bit), or when the
 * relaxation has not reached its fixed point after 16,384 launches (nothing is written then;
 * every launch moves the distance front across whole tiles, so real frames need a handful);
 * DGF_ERR_CAPACITY when a seed's cell touches more than 32 others or a neighbour search
 * holds more than 384 candidates (about 210 at k = 128 on dense grids; the outputs of the
 * affected cells are then NaN). */
int dgf_epic(const dgf_image *I0, const float *points, const float *flow, const uint8_t *status, int64_t n,
             const dgf_epic_opts *opts, void *workspace, size_t ws_bytes, float *dense, int64_t dense_pitch,
             int32_t *labels, uint32_t *dist, int32_t *nbr, uint32_t *nbr_dist, float *model, void *stream);

/* dgf_epic without host synchronisation, for graph capture and pipelines that must not stall the
 * host: the same computation and outputs, enqueued on `stream` with a fixed number of geodesic
 * relaxation launches, max_relax (0 = 32; at most 16,384).  A launch after one that changed
 * nothing returns at once, so launches beyond the fixed point cost a few microseconds each; the
 * ones dgf_epic needs are those a frame needs here (two to a dozen on 2048 x 1024 frames).
 * status_out (device uint32, 4-byte aligned) is written by the last kernel of the call: 0 done;
 * 1 the relaxation had not reached its fixed point after max_relax launches (the outputs are not
 * written: run again with more launches); 2 a capacity limit (DGF_ERR_CAPACITY of dgf_epic, with
 * its outputs).  The host-checked conditions of dgf_epic are returned as there
 * (DGF_ERR_INVALID_ARG also for a null or misaligned status_out or max_relax out of range). */
int dgf_epic_async(const dgf_image *I0, const float *points, const float *flow, const uint8_t *status, int64_t n,
                   const dgf_epic_opts *opts, void *workspace, size_t ws_bytes, float *dense, int64_t dense_pitch,
                   int32_t *labels, uint32_t *dist, int32_t *nbr, uint32_t *nbr_dist, float *model,
                   int32_t max_relax, uint32_t *status_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DEGRAF_FLOW_H */
