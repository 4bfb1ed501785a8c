/* tbr.h -- C ABI of the deposition-stroke renderer on MI355X (gfx950).
 *
 * The operations are those of "TBR: Transport-Based Rendering with
 * Deposition Strokes for Inverse Graphics" (arxiv 2609.08722):
 *   - a program of N capsule strokes, each with segment, half-width and a
 *     colour (Sec. 3, problem formulation; footprint K_i = closed capsule);
 *   - the per-pixel chain x_N = x, x_{i-1} = psi_i(x_i), with coverage
 *     evaluated at x_i, composited back to front (Sec. 3, Eq. chain and
 *     Eq. render), with psi_i the capsule insertion's backward map
 *     (Sec. 4, Eq. back, centred arclength, extension into the footprint,
 *     and the implemented floor C >= (eps r)^2 of Sec. 5.2);
 *   - hard coverage 1_{K_i} or the soft relaxation
 *     sigmoid((r - sigma) / max(tau r, tau_min)) (Sec. 5.1, Eq. relax),
 *     clamped at 1 - 1e-7 (Sec. 5.2);
 *   - the replay adjoint (Sec. 5.2: Eq. rpos, Eq. rT, the side table of
 *     positions where the floor binds, periodic checkpoints, Eq. adjstep
 *     and Eq. adjparam), and one Adam step of the inverse problem on the
 *     L2 data term (Sec. 3 Eq. inverse, Sec. 5.1 objective).
 *
 * Conventions shared by every call:
 *   - Pointers named as device pointers are HIP device memory owned by the
 *     caller; the library never allocates or frees device memory in these
 *     calls (workspaces are passed in, sized by the *_bytes queries).
 *   - Every call is ordered on the caller's hipStream_t `stream` (NULL = the
 *     legacy default stream) and is asynchronous unless stated otherwise.
 *   - Floats are IEEE FP32; images are row-major [H][W][3], pixel (i, j)
 *     sampled at its centre ((j + .5) / W, (i + .5) / H) of the canvas
 *     [0, 1]^2.
 *   - A stroke is (centre m = (cx, cy), angle phi, length L, half-width r):
 *     segment m +- (|L| / 2)(cos phi, sin phi); L = 0 is a drop. Its colour
 *     is c = softmax(z / tau_c) P over the palette P (tau_c = 0: P[argmax z]).
 *     The background is P[0].
 *   - Scalar arguments are validated on the host: a violation returns
 *     TBR_E_INVALID without launching anything, and tbr_last_error() says
 *     why. Device array contents are not inspected: NaN values or r <= 0
 *     give unspecified results (the device code is compiled assuming no
 *     NaN). Launch failures return TBR_E_DEVICE. No call aborts.
 *   - Calls are re-entrant given distinct workspaces.
 */
#ifndef TBR_H_
#define TBR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tbr_status {
  TBR_OK = 0,
  TBR_PENDING = 1,        /* serving: request not finished yet */
  TBR_E_INVALID = -1,     /* bad scalar argument, null pointer or short workspace */
  TBR_E_NOMEM = -2,       /* serving arena cannot ever hold the request */
  TBR_E_OVERFLOW = -3,    /* side table capacity exceeded (see tbr_tape_records) */
  TBR_E_CAPACITY = -4,    /* serving queue full */
  TBR_E_DEVICE = -5,      /* HIP runtime error */
  TBR_E_CANCELLED = -6,   /* serving: request cancelled */
  TBR_E_NOTFOUND = -7     /* serving: unknown ticket or program id */
} tbr_status;

/* Render modes (bit flags; both may be requested in one call). */
enum { TBR_HARD = 1, TBR_SOFT = 2 };

/* A stroke program (Sec. 3): device pointers, read-only.
 * cx, cy, angle, length, half_width: [n_strokes]; logits: [n_strokes * n_palette]
 * row-major; palette: [n_palette * 3] RGB, palette[0] is the background. */
typedef struct tbr_program {
  int32_t n_strokes;   /* N >= 0 */
  int32_t n_palette;   /* 1 <= K <= 64 */
  const float* cx;
  const float* cy;
  const float* angle;
  const float* length;
  const float* half_width;
  const float* logits;
  const float* palette;
} tbr_program;

/* Gradient outputs, same shapes as tbr_program's arrays (device, written). */
typedef struct tbr_program_grad {
  float* cx;
  float* cy;
  float* angle;
  float* length;
  float* half_width;
  float* logits;
  float* palette;
} tbr_program_grad;

/* Transport of a stroke (the insertion map every render, adjoint and fit
 * step applies).
 *   TBR_TRANSPORT_CAPSULE: the capsule insertion operator of Sec. 4
 *     (Eq. phi / Eq. back / Eq. fwd): every leaf of the area chart receives
 *     the area A_l(r) and the deposit is {sigma' <= r}.
 *   TBR_TRANSPORT_COUPLED: the calibrated variant of Sec. 4 ("A variant
 *     closer to line-source potential flow", Eq. coupling, Eq. profile): the
 *     leaf of centred arclength fraction v receives A_l(r) g(v), with
 *     g(v) = 1 + c_1 cos 4 pi v + c_2 cos 8 pi v + c_3 cos 12 pi v per
 *     stroke; the deposit is {u <= A_l(r) g(v)}, i.e. sigma' <= rl(v) with
 *     A_l(rl) = A_l(r) g(v). The hard footprint and the soft coverage
 *     sigmoid((rl(v) - sigma') / max(tau r, tau_min)) use that edge; the
 *     floor stays (eps r)^2. The coefficients are constants of the call:
 *     no gradient flows to them. g must be positive on every leaf (check a
 *     coefficient table with tbr_coupling_check); where it is not, the
 *     kernels take g = 0 and the result is meaningless.
 *   TBR_TRANSPORT_INERT: the inert-mark model R_U (Def. inert-mark): psi =
 *     id, each stroke composited where it is drawn. Renders, adjoint and fit
 *     steps; no side-table records are made.
 *   TBR_TRANSPORT_DROPS16: the renderer R_D the paper scores with (Sec.
 *     "Transfer across transport constructions"): capsule coverage, but the
 *     displacement is K = 16 drop maps (Lu 2012) of radius s, K pi s^2 =
 *     A_l(r), at the centres of 16 equal pieces of the segment, laid from its
 *     -e end (e = (cos angle, sin angle)) and undone last to first, each
 *     with the floor pi rho'^2 >= (eps s)^2. Renders, adjoint and fit steps:
 *     the tape's side table holds x_i wherever a drop's floor bound, and the
 *     replay regenerates through the drops' forward maps elsewhere. */
enum {
  TBR_TRANSPORT_CAPSULE = 0,
  TBR_TRANSPORT_COUPLED = 1,
  TBR_TRANSPORT_INERT = 2,
  TBR_TRANSPORT_DROPS16 = 3
};

typedef struct tbr_render_opts {
  int32_t width, height;  /* 1 .. 16384 each */
  float tau;              /* relative relaxation width, >= 0 (Eq. relax) */
  float tau_min;          /* absolute floor of the width, > 0 for soft renders */
  float tau_c;            /* colour temperature, >= 0 (0 = argmax colours) */
  float eps_floor;        /* floor constant eps of C >= (eps r)^2, > 0 (paper: 1e-3) */
  int32_t ckpt_interval;  /* position checkpoint interval k of the adjoint, >= 0 (0 = none) */
  int32_t side_slots;     /* per-pixel side-table capacity, >= 1 when a tape is written */
  int32_t transport;      /* a TBR_TRANSPORT_* value (0 = the capsule operator) */
  const float* coupling;  /* COUPLED: device [n_strokes * 3], (c_1, c_2, c_3) per stroke, read
                             by the call's stroke preparation; otherwise ignored (may be NULL) */
} tbr_render_opts;

/* ---------------------------------------------------------------------------
 * Closed-form compensation baseline (Sec. "Closed-form compensation
 * baseline", Table compensation, Lemma obstruction): an inert-mark program
 * is turned into one whose strokes, drawn under the capsule transport, land
 * where the inert program drew them. From the last stroke to the first, the
 * anchor a_i = m_i - (L_i / 2) e_i of stroke i (endpoint != 0: also its end
 * m_i + (L_i / 2) e_i) is pre-imaged through the backward maps of all later
 * strokes in their compensated geometry: N(N-1)/2 point maps (twice that for
 * the endpoint variant). The anchor variant keeps the offset L_i e_i; the
 * endpoint variant takes the segment between the two pre-images (angle kept
 * when they coincide). A step whose point lies in a later footprint (sigma'
 * <= r_j) is blocked: no pre-image exists; it is clamped by the extended map
 * with the floor (eps_floor r_j)^2, or left out (skip_blocked != 0).
 * ------------------------------------------------------------------------- */

/* Device workspace bytes of tbr_compensate (the pending points, FP64). */
size_t tbr_compensate_workspace_bytes(int32_t n_strokes, int32_t endpoint);

/* inert: the program (device). Outputs, device [n_strokes], written: the
 * compensated cx, cy, angle, length (half-widths, logits and palette are
 * unchanged) and the number of blocked steps of each stroke. eps_floor > 0.
 * One workgroup runs the N sequential steps on the stream. TBR_E_INVALID for
 * NULL outputs (allowed when n_strokes is 0), a bad program or a short
 * workspace. */
tbr_status tbr_compensate(const tbr_program* inert, float eps_floor, int32_t endpoint,
                          int32_t skip_blocked, float* cx, float* cy, float* angle, float* length,
                          int32_t* blocked, void* workspace, size_t workspace_bytes, void* stream);

/* Exact positivity check of the coupled profiles (Sec. 4: g is a cubic in
 * cos 4 pi v on [-1, 1], so its minimum is at an end or at a root of its
 * derivative). coupling: HOST [n_strokes * 3]. Writes the smallest value of
 * g over all strokes and leaves to *min_g (may be NULL; 1 when n_strokes is
 * 0). TBR_E_INVALID if it is not > 0 (or a coefficient is not finite). */
tbr_status tbr_coupling_check(const float* coupling, int32_t n_strokes, float* min_g);

/* Per-group Adam settings for tbr_fit_step (Sec. 5.1, Table hyper). */
typedef struct tbr_adam_opts {
  float lr_centre, lr_angle, lr_length, lr_width, lr_logits, lr_palette;
  float beta1, beta2, eps;
  float r_lo, r_hi;  /* half-width clamp after the update */
  float l_max;       /* |L| clamp after the update */
  int32_t step;      /* 1-based step index for bias correction */
} tbr_adam_opts;

/* Workspace bytes for tbr_render. With with_tape != 0 (soft mode only) the
 * workspace also holds the replay tape that tbr_render_backward consumes:
 * the final state s_0, checkpoints of (x, T) every ckpt_interval states and
 * the side table [side_slots][P] of positions where the floor bound. */
size_t tbr_render_workspace_bytes(const tbr_render_opts* opts, int32_t n_strokes, int32_t mode,
                                  int32_t with_tape);

/* Forward render (Eq. chain + Eq. render).
 * mode: TBR_SOFT and/or TBR_HARD.
 * rgb [H*W*3]: soft composite if TBR_SOFT is set, else the hard colour; may
 *   be NULL. label [H*W] (hard): palette index of the hard colour, 0 for
 *   background; owner [H*W] (hard): 0-based index of the stroke owning the
 *   pixel or -1; both may be NULL.
 * with_tape: record the replay tape into the workspace (requires TBR_SOFT).
 * Returns TBR_OK once launched; a side-table overflow is only detectable
 * with tbr_tape_records. */
tbr_status tbr_render(const tbr_program* prog, const tbr_render_opts* opts, int32_t mode,
                      float* rgb, int32_t* label, int32_t* owner, void* workspace,
                      size_t workspace_bytes, int32_t with_tape, void* stream);

/* Allocation-free forward render, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): tbr_render without a tape and without a workspace
 * argument. The prepared stroke records (and the coupled transport's profile
 * coefficients) go to a 1 MiB array that the library holds in device memory,
 * one per device, until the process ends; the call itself allocates nothing
 * and calls no allocating routine. Arguments, outputs and results are those
 * of tbr_render(prog, opts, mode, rgb, label, owner, ws, ws_bytes, 0, stream),
 * bitwise. TBR_E_CAPACITY if n_strokes > TBR_STATIC_MAX_STROKES. Every call
 * on one device shares that device's array: calls whose executions overlap
 * on one device (different streams, or other host threads) race and give
 * undefined results; calls ordered on one stream do not. */
#define TBR_STATIC_MAX_STROKES 8192
tbr_status tbr_render_static(const tbr_program* prog, const tbr_render_opts* opts, int32_t mode,
                             float* rgb, int32_t* label, int32_t* owner, void* stream);

/* Largest number of side-table records any pixel needed in the last taped
 * render of this workspace. SYNCHRONISES the stream. Returns TBR_E_OVERFLOW
 * when it exceeds opts->side_slots (the tape is then incomplete and the
 * render must be repeated with at least *max_records slots). */
tbr_status tbr_tape_records(const void* workspace, size_t workspace_bytes,
                            const tbr_render_opts* opts, int32_t n_strokes,
                            int32_t* max_records, void* stream);

/* Workspace bytes for tbr_render_backward (per-tile partial rows of the
 * deterministic gradient reduction). */
size_t tbr_backward_workspace_bytes(const tbr_render_opts* opts, int32_t n_strokes,
                                    int32_t n_palette);

/* Replay adjoint of the soft render (Sec. 5.2): vector-Jacobian product of
 * the rendered image with grad_rgb [H*W*3] (dL/dR), written to every array
 * of *grad (overwritten, not accumulated). tape_ws is the workspace of the
 * preceding tbr_render(..., TBR_SOFT, ..., with_tape = 1) of the same
 * program and options. Deterministic: no atomics, fixed summation order. */
tbr_status tbr_render_backward(const tbr_program* prog, const tbr_render_opts* opts,
                               const void* tape_ws, size_t tape_bytes, const float* grad_rgb,
                               const tbr_program_grad* grad, void* workspace,
                               size_t workspace_bytes, void* stream);

/* Workspace bytes for tbr_fit_step (tape + reduction + gradients). */
size_t tbr_fit_workspace_bytes(const tbr_render_opts* opts, int32_t n_strokes,
                               int32_t n_palette);

/* One optimisation step of the inverse problem with the pixel L2 data term
 * L = mean((R - I*)^2) over the 3 H W values: soft render with tape, seed
 * dL/dR, replay adjoint, deterministic reduction, and an Adam update. The
 * render, seed and replay of each 16x16 tile run back to back in one
 * persistent launch (the kernel of tbr_fit_multi_step with one job); the
 * results equal tbr_render + tbr_render_backward with that seed bitwise.
 * params: packed device vector [cx N | cy N | angle N | length N |
 *   half_width N | logits N*K | palette K*3], updated in place.
 * grads: same layout, written (may be NULL: kept in the workspace).
 * adam_m, adam_v: Adam moments, same layout, updated in place.
 * target_rgb [H*W*3]; loss: device scalar, written (value before the update).
 * Half-width is clamped to [r_lo, r_hi], |length| to l_max, palette to [0,1].
 * Side-table overflow (some pixel needed more than opts->side_slots records)
 * is checked on the device before the update: the step then leaves params,
 * adam_m and adam_v unchanged (grads and loss are written but describe an
 * incomplete adjoint), and tbr_tape_records on this workspace reports
 * TBR_E_OVERFLOW with the needed count. Growing side_slots and calling the
 * step again repeats it exactly. */
tbr_status tbr_fit_step(int32_t n_strokes, int32_t n_palette, float* params, float* grads,
                        float* adam_m, float* adam_v, const tbr_adam_opts* adam,
                        const tbr_render_opts* opts, const float* target_rgb, float* loss,
                        void* workspace, size_t workspace_bytes, void* stream);

/* One job of a batched fit: its own program (packed params, as in
 * tbr_fit_step), Adam state, target, options and step settings. */
typedef struct tbr_fit_job {
  int32_t n_strokes, n_palette;
  float* params;            /* packed [cx|cy|angle|length|half_width|logits|palette], in place */
  float* grads;             /* packed gradient, written (may be NULL) */
  float* adam_m;
  float* adam_v;
  const float* target_rgb;  /* [H*W*3] */
  float* loss;              /* device scalar, written */
  tbr_render_opts opts;
  tbr_adam_opts adam;
} tbr_fit_job;

/* Workspace bytes for tbr_fit_multi_step over these jobs (1..16 jobs). */
size_t tbr_fit_multi_workspace_bytes(const tbr_fit_job* jobs, int32_t n_jobs);

/* One fit step (as tbr_fit_step) for every job, with the soft forward and
 * the replay adjoint of ALL jobs fused into one persistent launch: blocks
 * take (job, 16x16 tile) items, largest jobs first, and per tile run the
 * forward with tape, the L2 seed and the replay of that tile. Reductions and
 * Adam follow per job. Each job's results equal its own tbr_fit_step
 * (partial rows are indexed by tile, so the summation order is fixed). */
tbr_status tbr_fit_multi_step(const tbr_fit_job* jobs, int32_t n_jobs, void* workspace,
                              size_t workspace_bytes, void* stream);

/* Side-table high-water marks of the last multi step, per job
 * (max_records[n_jobs]). SYNCHRONISES the stream; TBR_E_OVERFLOW if any job
 * overflowed its side_slots. A job that overflowed had its update skipped,
 * as in tbr_fit_step; the other jobs were updated. */
tbr_status tbr_fit_multi_records(const tbr_fit_job* jobs, int32_t n_jobs, const void* workspace,
                                 size_t workspace_bytes, int32_t* max_records, void* stream);

/* ---------------------------------------------------------------------------
 * Fitting loop (Sec. 5.1 "Parameterisation and relaxation", Table hyper,
 * Sec. 8 "Area budget"). The optimiser works on unconstrained free
 * parameters theta, packed like the program:
 *   [th_ax N | th_ay N | th_dx N | th_dy N | th_r N | th_c N*K | th_P K*3].
 * Windows map them to the program: anchor a = a_lo + (a_hi - a_lo)
 * sigmoid(th_a) and offset d = l_max tanh(th_d), each per component; the
 * stroke runs from a to a + d, so m = a + d / 2, L = |d| and
 * phi = atan2(d_y, d_x) (0 when d = 0); half-width
 * r = (r_lo_frac + (r_hi_frac - r_lo_frac) sigmoid(th_r)) r0_i with r0_i
 * geometric from r0_first (stroke 0) to r0_last (stroke N-1); logits
 * z = th_c; palette P = sigmoid(th_P).
 * ------------------------------------------------------------------------- */
typedef struct tbr_window_opts {
  float a_lo, a_hi;            /* anchor window, a_hi > a_lo (the paper's: the canvas, 0 and 1) */
  float l_max;                 /* offset bound per component, > 0 (Table hyper: 0.30) */
  float r0_first, r0_last;     /* > 0 (Table hyper: 0.120 and 0.005) */
  float r_lo_frac, r_hi_frac;  /* 0 < lo < hi (Table hyper: 0.6 and 1.7) */
  float lambda_length;         /* lambda sum_i |L_i| (Table hyper: 3e-4), >= 0 */
  float lambda_area;           /* lambda_A sum_i A_l(r_i), >= 0 */
} tbr_window_opts;

/* params = window map of theta (device, packed as above / as the program).
 * TBR_E_INVALID for out-of-range sizes or window options. */
tbr_status tbr_window_map(int32_t n_strokes, int32_t n_palette, const float* theta, float* params,
                          const tbr_window_opts* window, void* stream);

/* One step of the fitting loop: params = window map of theta; the fit step's
 * soft render, L2 seed and replay adjoint (workspace as
 * tbr_fit_workspace_bytes) give the data loss and its gradient w.r.t. the
 * program (written to grads, or kept in the workspace if NULL); *loss gets
 * the data loss plus lambda sum |L| + lambda_A sum A_l(r); the gradient of
 * that total is chained through the windows and theta takes one Adam step
 * with the group steps lr_centre (anchor), lr_length (offset), lr_width
 * (half-width), lr_logits (colour) and lr_palette (palette); lr_angle and
 * the clamps of tbr_adam_opts are not used. The step's tau and tau_c come
 * from opts (see tbr_schedule_at). A side-table overflow skips the update
 * as in tbr_fit_step. */
tbr_status tbr_fit_loop_step(int32_t n_strokes, int32_t n_palette, float* theta, float* params,
                             float* grads, float* adam_m, float* adam_v,
                             const tbr_window_opts* window, const tbr_adam_opts* adam,
                             const tbr_render_opts* opts, const float* target_rgb, float* loss,
                             void* workspace, size_t workspace_bytes, void* stream);

/* The schedule of Table hyper at step s of total_steps (host only):
 * tau and tau_c geometric from first (s = 0) to last (s = total_steps - 1),
 * and the cosine step factor (1 + cos(pi s / total_steps)) / 2. */
void tbr_schedule_at(int32_t step, int32_t total_steps, float tau_first, float tau_last,
                     float tau_c_first, float tau_c_last, float* tau, float* tau_c,
                     float* lr_scale);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of replay requests (the forward render above,
 * for many programs, resolutions and modes arriving over time).
 *
 * A server owns a scheduler thread and a set of HIP streams (default
 * priority). Programs are registered once and copied into the caller's
 * device arena, where they stay resident. Each scheduler tick:
 *   1. retires launches that finished, freeing their requests' slots and
 *      arena bytes;
 *   2. admits queued requests in FIFO order while a slot is free and the
 *      arena can hold the request's HBM footprint: its prepared stroke
 *      records (tbr_serve_request_bytes) plus the outputs it asks the server
 *      to hold in the arena (tbr_serve_output_bytes);
 *   3. packs the admitted requests into one persistent launch over
 *      (request, 16x16 tile) work items; the requests of a launch retire
 *      together, so one of at least solo_tiles tiles gets a launch of its
 *      own.
 * Each stream owns a hipGraph built at create time: one copy of the tick's
 * descriptors and work list from pinned host staging, a kernel that clears
 * the work cursor, one stroke-preparation launch for all of the tick's
 * requests and the persistent render launch. A tick updates the copy size
 * and the launches' grids and arguments, then launches the graph.
 * Launches rotate over `streams` streams, so requests admitted while others
 * run overlap with them on the device. Every pixel is computed by the same
 * device code as tbr_render, so a request's result does not depend on what
 * else is in flight. An output is either caller memory, which must stay valid
 * until the ticket completes, or held by the server in the arena
 * (tbr_request.arena_outputs): then it counts towards the request's
 * footprint from admission, its address comes with the completed poll, and
 * it stays valid (its bytes stay taken) until tbr_serve_release.
 * ------------------------------------------------------------------------- */
typedef struct tbr_server tbr_server;

typedef struct tbr_serve_opts {
  void* arena;                    /* device memory owned by the caller (NULL only with fake_device) */
  size_t arena_bytes;             /* programs + admitted requests + per-stream launch buffers */
  int32_t max_slots;              /* requests admitted (in flight) at once, >= 1 */
  int32_t max_queue;              /* requests waiting for admission, >= 1 */
  int32_t max_tick_items;         /* (request, tile) work items per launch, >= 1 */
  int32_t streams;                /* launches in flight at once, 1..4 */
  int32_t fake_device;            /* 1: host-only executor for scheduler tests; no GPU work */
  float fake_ns_per_pixel_stroke; /* fake executor: modelled cost per pixel-stroke */
  int32_t fake_fail_launch;       /* fake executor: the 1-based launch that reports a device
                                     error on completion (0: none); ignored on a GPU */
  int32_t solo_tiles;             /* a request of at least this many 16x16 tiles runs in a
                                     launch of its own (0: every request may share one) */
} tbr_serve_opts;

/* Outputs of a request that the server holds in its arena. */
enum { TBR_OUT_RGB = 1, TBR_OUT_LABEL = 2, TBR_OUT_OWNER = 4, TBR_OUT_ALL = 7 };

typedef struct tbr_request {
  uint64_t program_id;            /* from tbr_serve_register_program */
  int32_t mode;                   /* TBR_SOFT or TBR_HARD */
  int32_t width, height;          /* 1 .. 16384 */
  float tau, tau_min, tau_c, eps_floor;  /* as tbr_render_opts; tau_min <= 0 means
                                            (float)(0.7 / (double)width) */
  float* rgb;                     /* device [H*W*3]: soft composite, or hard colour (may be NULL for hard) */
  int32_t* label;                 /* hard: device [H*W] or NULL */
  int32_t* owner;                 /* hard: device [H*W] or NULL */
  int32_t arena_outputs;          /* TBR_OUT_* mask of outputs held in the arena by the server
                                     (their pointers above must be NULL; soft: TBR_OUT_RGB only) */
} tbr_request;

typedef struct tbr_result {
  int32_t status;                 /* TBR_OK, TBR_PENDING, TBR_E_CANCELLED or TBR_E_DEVICE */
  double t_submit, t_admit, t_start, t_done;  /* seconds on tbr_serve_now()'s clock */
  int64_t pixel_strokes;          /* width * height * n_strokes */
  float* rgb;                     /* the request's outputs (device): the caller's pointers, or */
  int32_t* label;                 /* for TBR_OUT_* ones the arena addresses once complete, */
  int32_t* owner;                 /* valid until tbr_serve_release */
} tbr_result;

typedef struct tbr_serve_stats {
  int64_t submitted, completed, cancelled, launches;
  int64_t pixel_strokes;          /* of completed requests */
  int64_t queued, in_flight;
  size_t arena_used, arena_bytes;
} tbr_serve_stats;

/* Arena bytes of one resident program, of one admitted request, and of the
 * per-stream launch buffers (descriptors, preparation descriptors, work list
 * and cursor; the arena must hold streams * tick bytes plus the programs
 * plus the in-flight requests). */
size_t tbr_serve_program_bytes(int32_t n_strokes, int32_t n_palette);
size_t tbr_serve_request_bytes(int32_t n_strokes);
size_t tbr_serve_tick_bytes(const tbr_serve_opts* opts);
/* Arena bytes of the outputs a request asks the server to hold (a TBR_OUT_*
 * mask): 12 B per pixel for rgb, 4 B each for label and owner. 0 for a bad
 * canvas or mask. */
size_t tbr_serve_output_bytes(int32_t width, int32_t height, int32_t arena_outputs);

/* Create a server (starts its scheduler thread). */
tbr_status tbr_serve_create(const tbr_serve_opts* opts, tbr_server** server);

/* Copy a program (device arrays) into the arena; synchronous. TBR_E_NOMEM
 * when the arena cannot hold it. */
tbr_status tbr_serve_register_program(tbr_server* server, const tbr_program* program,
                                      uint64_t* program_id);

/* Queue a request; returns at once with a ticket. TBR_E_CAPACITY when the
 * queue is full, TBR_E_NOMEM when the request's footprint exceeds the arena
 * less its launch buffers and programs (it could never be admitted),
 * TBR_E_NOTFOUND for an unknown program, TBR_E_INVALID for a bad canvas,
 * relaxation, mode, output set or arena_outputs mask. */
tbr_status tbr_serve_submit(tbr_server* server, const tbr_request* request, uint64_t* ticket);

/* TBR_OK (request finished; its outputs are complete on the device),
 * TBR_E_CANCELLED, or TBR_E_DEVICE (its launch failed), after which the ticket
 * is forgotten, except that a finished request holding arena outputs keeps
 * them (and its ticket) until tbr_serve_release; TBR_PENDING while queued or
 * running. Fills *result in every case. Does not synchronise. */
tbr_status tbr_serve_poll(tbr_server* server, uint64_t ticket, tbr_result* result);

/* Give back a finished request's arena outputs (and forget its ticket) once
 * the caller has consumed them: work of the caller's that reads them must be
 * complete, since the bytes may be handed to the next admitted request at
 * once. TBR_OK; TBR_PENDING while the request is queued or running;
 * TBR_E_NOTFOUND for an unknown or forgotten ticket. */
tbr_status tbr_serve_release(tbr_server* server, uint64_t ticket);

/* Cancel a queued request (TBR_OK); an admitted one runs to completion
 * (TBR_PENDING). */
tbr_status tbr_serve_cancel(tbr_server* server, uint64_t ticket);

tbr_status tbr_serve_get_stats(tbr_server* server, tbr_serve_stats* stats);

/* Stop the scheduler, wait for launches in flight, free host resources. */
void tbr_serve_destroy(tbr_server* server);

/* The serving clock (steady, seconds). */
double tbr_serve_now(void);

/* Optional timing hook for benchmarks. While set on the calling thread,
 * every launch of the kernel named `kernel` ("trace_soft", "trace_hard",
 * "replay" or "fit_fused") made by a tbr_* call on this thread is bracketed by
 * hipEventRecord(begin) / hipEventRecord(end) on that call's stream (with
 * several launches, the last pair stands). begin and end are hipEvent_t
 * handles owned by the caller. kernel = NULL clears the hook. */
tbr_status tbr_set_timing_events(const char* kernel, void* begin, void* end);

/* Thread-local description of the last non-OK status of this thread. */
const char* tbr_last_error(void);

/* Library version string. */
const char* tbr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TBR_H_ */
