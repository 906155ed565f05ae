/*
 * fd.h -- C ABI of libfd, an MI355X (gfx950) finite-difference stepper for
 * the second-order acoustic wave equation with a damping layer, off-grid
 * point sources and receivers, its exact discrete adjoint and the
 * imaging-condition gradient, plus a continuous-batching shot server.
 *
 * The calls follow the way the thesis states a finite-difference problem
 * (Section 2.1.1): a Grid with a shape and an extent, a TimeFunction with a
 * time order and a space order (time order is 2 here), a Function for the
 * medium, SparseTimeFunctions for sources and receivers, and an Operator
 * applied for nt steps with a time step dt.  Sources and receivers are the
 * per-step work that its GPU backend could not own (Section 6.2.1); here they
 * run on the device inside the step.  Datasets are reached through opaque
 * handles as in the structured-mesh API of Section 2.2, but -- unlike that
 * API, which takes ownership of the data -- the caller owns every device
 * buffer: the library sizes a workspace, borrows it, and never frees it.
 *
 * Equations (readings of the thesis; the stepper is the centred leapfrog):
 *   m u_tt + m sigma u_t - Lap_h u = q,   m = 1/v^2
 *   u^{n+1} = [2u^n - (1 - sigma dt/2) u^{n-1} + dt^2 v^2 (Lap_h u^n + q^n)]
 *             / (1 + sigma dt/2)
 *   Lap_h: maximal-order central 2nd-derivative weights of space order so
 *   (radius r = so/2 per axis, star stencil of Section 3.3.3), the field
 *   taken as zero outside the padded grid.
 *   sigma(i) = damp_max * sum_a (d_a/nbl)^2, d_a = distance into the layer.
 *   q^n = sum_s w_s[n] W_s / prod(h)  (multilinear weights W over the 2^d
 *   corners of the cell holding the source); rec_r[n] = sum W_r u^{n+1}.
 *   With sinc_radius r > 0, W is instead the tensor product over axes of
 *   Kaiser-windowed sinc weights on the 2r nodes around the point (Hicks,
 *   Geophysics 67(1), 2002): for a node at signed distance x (in cells),
 *   sinc(x) I0(b sqrt(1 - (x/r)^2)) / I0(b); nodes outside the padded grid
 *   are dropped (the field is zero there).  Injection stays the transpose
 *   of interpolation, so the adjoint below stays exact.
 *
 * Conventions shared by every call:
 *   - Return FD_OK (0) or a negative fd_status; fd_last_error() gives a
 *     thread-local message.  No C++ exception crosses the ABI.
 *   - "device" pointers are HIP device pointers on the device current when
 *     the grid was created; "host" pointers are ordinary host memory read
 *     before the call returns.
 *   - Calls taking a stream (hipStream_t passed as void*, NULL = the null
 *     stream) enqueue their work and return without synchronising, unless
 *     stated otherwise; device errors raised by enqueued work surface as
 *     FD_ERR_DEVICE on a later call.  Calls on one grid must be ordered on
 *     one stream (they share the grid's wavefield buffers).
 *   - Dense padded fields (initial/final states, gradients) are C arrays
 *     [Nz'][Ny'][Nx'] (3D) or [Nz'][Nx'] (2D), x fastest, N' = N + 2 nbl.
 *   - Coordinates are metres in grid axis order: (x, y, z) or (x, z);
 *     a coordinate outside [origin, origin + (N-1) h] gives FD_ERR_ARG.
 */
#ifndef FD_H
#define FD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 2: fd_grid_desc gained param_storage and fd_grid_info the parameter
   fields (appended; zero-initialised descriptors keep the former behaviour,
   but callers built against version 1 pass the shorter structs and must be
   rebuilt) */
#define FD_API_VERSION 2

typedef enum fd_status {
    FD_OK = 0,
    FD_ERR_ARG = -1,       /* invalid argument or descriptor */
    FD_ERR_UNSTABLE = -2,  /* dt at or above the von Neumann limit */
    FD_ERR_NOMEM = -3,     /* workspace too small / HBM budget exceeded */
    FD_ERR_DEVICE = -4,    /* a HIP call or an enqueued kernel failed */
    FD_ERR_STATE = -5,     /* call not valid in the object's state */
    FD_ERR_TIMEOUT = -6    /* fd_wait timed out */
} fd_status;

typedef enum fd_storage {
    FD_STORE_F32 = 0,      /* float32 wavefields */
    FD_STORE_F16 = 1,      /* IEEE half wavefields (scaled by amp_scale), FP32 arithmetic */
    FD_STORE_BF16 = 2,     /* bfloat16 wavefields, FP32 arithmetic */
    /* 16-bit value and difference (3D only; fd_forward and the server, the
       adjoint stores two levels): u^n and u^n - u^{n-1} are kept instead of
       two levels, so the difference -- what the leapfrog update advances --
       keeps 16-bit relative precision where the time step is small against
       the local period; 12 B per point-step instead of 10, three 16-bit
       buffers */
    FD_STORE_F16_DIFF = 3,
    FD_STORE_BF16_DIFF = 4
} fd_storage;

/* Storage of the parameter p = dt^2 v^2 that multiplies the Laplacian in the
   update above.  It is read once per point-step: 4 of the 16 bytes of a
   float32 step.  A storage form of this library, not of the thesis. */
typedef enum fd_param_storage {
    FD_PARAM_F32 = 0,      /* float32 p, rounded once from dt^2 v^2 */
    /* 16-bit code of p on a uniform scale between its extremes: p0 =
       dt^2 v_min^2 and dp = dt^2 (v_max^2 - v_min^2) / 65535, both rounded to
       float32; code = the nearest integer in [0, 65535] to (p - p0) / dp,
       evaluated in float64 from p = dt^2 v^2; the step uses
       fma(code, dp, p0) in float32.  Any velocity range fits, and a point's
       p moves by at most dp / 2 plus one float32 rounding (relative: 2^-17
       (v_max^2 - v_min^2) / v_min^2, 6e-5 for 1.5-4.5 km/s): a fixed
       perturbation of the medium, not an error that grows with the steps.
       The step then moves 14 B per point-step with float32 wavefields, 8 B
       with two 16-bit levels and 10 B with the 16-bit value and difference.
       3D fd_forward, fd_adjoint and the server; fd_gradient refuses it, and
       two levels per launch are not available with it. */
    FD_PARAM_Q16 = 1
} fd_param_storage;

/* Grid description (Devito Grid + TimeFunction, Section 2.1.1). */
typedef struct fd_grid_desc {
    int ndim;              /* 2 or 3 */
    int shape[3];          /* physical points per axis, (x, y, z) or (x, z); each >= 2 */
    double spacing[3];     /* h per axis, metres, > 0 */
    double origin[3];      /* coordinate of the first physical point */
    int space_order;       /* even, 2..16 (stencil radius so/2) */
    int nbl;               /* damping-layer points added on every face, >= 0 */
    double damp_max;       /* sigma_max in 1/s; <= 0 selects 3 v_max ln(1000) / (2 nbl h_min) */
    int storage;           /* fd_storage */
    float amp_scale;       /* 16-bit storage keeps amp_scale * u; 0 selects 1 for BF16 and,
                              for F16, the power of two nearest prod(h)/(dt^2 v_max^2)
                              (the difference storages scale both fields alike) */
    int vp_padded;         /* 0: vp given on the physical grid, layer filled by edge
                              replication; 1: vp given on the padded grid */
    int max_src;           /* capacity of the source table (points), 0 selects 64 */
    int max_rec;           /* capacity of the receiver table (points), 0 selects 4096 */
    int zchunk;            /* planes marched per workgroup in 3D (at most 512, larger values are
                              clamped), 0 selects automatically */
    int sinc_radius;       /* 0: multilinear sparse weights; 1..8: Kaiser-windowed sinc
                              over (2 sinc_radius)^ndim nodes per point (the sparse
                              tables, about 36 B per node, scale with max_src and
                              max_rec: 3D radius 8 with 4096 receivers is 0.6 GB) */
    double sinc_beta;      /* Kaiser shape b; <= 0 selects pi * sinc_radius / 2 */
    int tile_x;            /* 3D workgroup tiles: 64 (64 x 16 xy tiles), 32 (32 x 32), 96
                              (64 x 16, and 32 x 32 for a last x column of at most 32
                              points; 64 x 16 alone when there is none; space orders 14
                              and 16 run 32 x 32 instead), 0 selects automatically; any
                              other value is FD_ERR_ARG; ignored in 2D */
    int time_block;        /* time steps per launch of fd_forward and the server: 1 one
                              step per launch; 2 two leapfrog levels per launch (3D,
                              float32 storage, space order <= 8 only: 64 x 16 tiles
                              whatever tile_x says, two more wavefield buffers in the
                              workspace); 0 selects automatically (two levels at space
                              order 2 in 3D float32, measured 11-12 % faster there; one
                              step elsewhere, where the recomputed ring of the two-level
                              kernel costs more than the traffic it saves); anything
                              else, or 2 where it is not available, is FD_ERR_ARG */
    int param_storage;     /* fd_param_storage; FD_PARAM_Q16 in 3D only */
} fd_grid_desc;

/* Sources and receivers of one shot (Devito SparseTimeFunction, Section 2.1.1). */
typedef struct fd_shot {
    int nsrc;                  /* >= 0 for fd_forward and fd_adjoint (0: nothing injected,
                                  an initial-value problem; src pointers may be NULL);
                                  >= 1 for fd_gradient and fd_submit */
    const double *src_xyz;     /* host, [nsrc][ndim] */
    const float *src_wavelet;  /* device, [nt][nsrc]; row n enters u^{n+1} */
    int nrec;                  /* >= 0 for fd_forward and fd_adjoint (0: no traces; rec
                                  pointers may be NULL); >= 1 for fd_gradient and fd_submit */
    const double *rec_xyz;     /* host, [nrec][ndim] */
} fd_shot;

/* Optional state for fd_forward (all device, dense padded float32, nullable). */
typedef struct fd_fwd_opts {
    const float *u0;       /* u^0 (NULL: zero) */
    const float *u_prev;   /* u^{-1} (NULL: zero) */
    float *save_u;         /* receives u^{nt} */
    float *save_u_prev;    /* receives u^{nt-1} */
} fd_fwd_opts;

/* Read-only facts about a created grid. */
typedef struct fd_grid_info {
    int ndim;
    int padded[3];         /* N' per axis (x, y, z) or (x, z) */
    long long padded_points;
    double vmax;           /* max velocity over the padded grid, m/s */
    double critical_dt;    /* von Neumann limit of the undamped update */
    double damp_max;       /* sigma_max in use, 1/s */
    size_t field_bytes;    /* one wavefield buffer as laid out on the device */
    int tile[2];           /* 3D: xy tile of the step workgroups in points (64 x 16 or
                              32 x 32); 2D: (64, 64), x points and z rows */
    int tile_strip;        /* 3D: width of the last x column when it runs 32 x 32 tiles
                              beside 64 x 16 ones, else 0 */
    int zchunk;            /* 3D: z planes per workgroup of a plain step; 2D: 64 */
    int time_block;        /* steps per launch of fd_forward (1 or 2) */
    int param_storage;     /* fd_param_storage in use */
    double param_base;     /* FD_PARAM_Q16: p0 and dp of the latest dt (float32 values), */
    double param_step;     /* 0 before the first call that steps or with FD_PARAM_F32 */
} fd_grid_info;

typedef struct fd_grid fd_grid;

/*
 * Bytes of device workspace fd_grid_create needs for this description.
 * Returns FD_ERR_ARG for an invalid description.
 */
int fd_grid_workspace_bytes(const fd_grid_desc *desc, size_t *bytes);

/*
 * Create a grid on the current device.  workspace: device buffer of at least
 * fd_grid_workspace_bytes(desc) bytes, 256-byte aligned, borrowed until
 * fd_grid_destroy.  vp_dev: device float32 velocity in m/s, dense, physical
 * or padded shape per desc->vp_padded, all values > 0; read during the call.
 * Synchronises `stream` once (to learn v_max).  *out receives the handle.
 */
int fd_grid_create(const fd_grid_desc *desc, void *workspace, size_t ws_bytes,
                   const float *vp_dev, void *stream, fd_grid **out);

/* Release the handle (host memory only; the workspace stays the caller's).
 * Waits for the work last enqueued on the grid (its latest stream) first. */
int fd_grid_destroy(fd_grid *grid);

/* Fill *info with the facts above (host only; FD_ERR_ARG on a null argument). */
int fd_grid_get_info(const fd_grid *grid, fd_grid_info *info);

/*
 * Forward modelling: the Operator applied for nt time steps with step dt
 * (Section 2.1.1; one launch per step from the host time loop, Section
 * 3.3.2), from u^0, u^{-1} (zero unless opts says otherwise).
 * rec_out: device float32 [nt][nrec], row n = receivers sampling u^{n+1}.
 * opts may be NULL; nt = 0 only applies opts (state in, state out).
 * Source and receiver tables are rebuilt on the host when the coordinates
 * differ from the previous call's.  Errors: FD_ERR_UNSTABLE if dt >=
 * critical_dt; FD_ERR_ARG for nt < 0, a null required pointer, a point
 * outside the grid or more points than max_src / max_rec; FD_ERR_DEVICE if
 * a HIP call fails.  A rejected call leaves the grid usable.
 */
int fd_forward(fd_grid *grid, const fd_shot *shot, int nt, double dt,
               float *rec_out, const fd_fwd_opts *opts, void *stream);

/*
 * Adjoint modelling (the exact transpose of fd_forward for a fixed medium,
 * zero initial state): residual_dev [nt][nrec] device float32 is injected at
 * the receivers backwards in time; src_adj_dev [nt][nsrc] device float32
 * receives (F^T r)_s[n] = dt^2/prod(h) sum_c W_s,c lambda^n.  The same step
 * kernel runs with the roles of sources and receivers exchanged.  Errors as
 * for fd_forward.
 *
 * The thesis motivates its stencil work by seismic inversion (Chapter 1,
 * Section 2.1), which needs this adjoint of the modelling operator; it
 * gives no formula for it.  The reading here is discretise-then-transpose:
 * starting from lambda^{nt} = lambda^{nt+1} = 0, for k = nt .. 1,
 *   lambda^{k-1} = [2 lambda^k - (1 - sigma dt/2) lambda^{k+1}
 *                   + dt^2 v^2 Lap_h lambda^k + v^2 P_r^T r^{k-1}] / (1 + sigma dt/2),
 * the exact transpose of the forward recursion, sources and receivers
 * above, so <F w, r> = <w, F^T r> holds to rounding.
 */
int fd_adjoint(fd_grid *grid, const fd_shot *shot, int nt, double dt,
               const float *residual_dev, float *src_adj_dev, void *stream);

/* Flags for fd_gradient. */
#define FD_GRAD_RESIDUAL_GIVEN 1   /* d_obs_dev holds the residual itself */
#define FD_GRAD_BINOMIAL 2         /* checkpoint_every is a number of snapshot slots (>= 0);
                                      the reverse sweep follows fd_checkpoint_schedule */
#define FD_GRAD_VELOCITY 4         /* grad_m_dev receives the gradient with respect to the
                                      velocity, g_v = g_m dm/dv = -2 g_m / v^3, with v the
                                      grid's padded velocity (sigma held fixed) */

/* Device workspace for fd_gradient.  Default: checkpoints of (u^c, u^{c-1})
 * every checkpoint_every steps except the last segment's (ceil(nt /
 * checkpoint_every) - 1 pairs) and checkpoint_every bracket fields of the
 * segment recompute; with checkpoint_every >= nt, nt bracket fields and no
 * checkpoint (the forward pass keeps every bracket, nothing is recomputed).
 * FD_GRAD_BINOMIAL: checkpoint_every + 1 snapshots and two scratch fields.
 * All add the float64 gradient, its float32 partial sum, traces and
 * residual. */
int fd_gradient_workspace_bytes(const fd_grid *grid, int nt, int nrec,
                                int checkpoint_every, int flags, size_t *bytes);

/* Actions of a binomial checkpoint schedule (host only, no device work). */
typedef enum fd_ckpt_kind {
    FD_ACT_ADVANCE = 1,   /* `count` forward steps from level `step` */
    FD_ACT_STORE = 2,     /* snapshot of the state at level `step` into `slot` */
    FD_ACT_RESTORE = 3,   /* make the state of `slot` (level `step`) current */
    FD_ACT_YOUTURN = 4    /* forward step `step` with its imaging bracket, then the
                             adjoint step producing lambda^step */
} fd_ckpt_kind;

typedef struct fd_ckpt_action {
    int kind;     /* fd_ckpt_kind */
    int step;     /* time level the action starts from */
    int count;    /* steps (ADVANCE), 1 (YOUTURN), 0 otherwise */
    int slot;     /* snapshot slot (STORE, RESTORE; 0 holds the initial state) */
    int first;    /* 1 if the action computes some step for the first time */
} fd_ckpt_action;

/*
 * Schedule reversing nt steps with `slots` snapshot slots besides the initial
 * state, minimising the number of forward steps (binomial checkpointing,
 * Griewank-Walther: the smallest optimal split of each segment, found by
 * bisection on the closed-form cost; host time and memory grow with the
 * number of actions only).  Writes up to `capacity` actions (actions may be
 * NULL to query the count), the count to *n_actions and the ADVANCE steps to
 * *forward_steps (nullable).  FD_ERR_ARG for nt < 1, slots < 0 or nt above
 * INT_MAX / 8.
 */
int fd_checkpoint_schedule(int nt, int slots, fd_ckpt_action *actions, int capacity,
                           int *n_actions, long long *forward_steps);

/*
 * Misfit and gradient for seismic inversion, the application the thesis's
 * stencil work serves (Chapter 1, Section 2.1); the thesis states neither
 * the misfit nor the imaging condition, so the reading is the exact
 * derivative of the discrete forward map above (discretise-then-
 * differentiate).  Gradient with respect to m = 1/v^2 on the padded grid
 * (or v with FD_GRAD_VELOCITY), sigma held fixed (all checkpointing modes
 * give bitwise the same result):
 *   J = 1/2 sum_n sum_r (rec_r[n] - d_obs_r[n])^2
 *   g_m = - sum_n lambda^n [(u^{n+1} - 2u^n + u^{n-1}) + (sigma dt/2)(u^{n+1} - u^{n-1})]
 * with lambda the adjoint field driven by the residual.  The bracket of each
 * level comes from a forward step that also writes it: recomputed from
 * checkpoints, or kept from the forward pass (the last segment's levels,
 * and every level when checkpoint_every >= nt).
 * Products are summed in float32 over 32 adjoint steps, then added to the
 * float64 gradient.  d_obs_dev: device float32 [nt][nrec]
 * (the residual itself when flags has FD_GRAD_RESIDUAL_GIVEN).
 * misfit_dev: device double[1]; grad_m_dev: device double, dense padded;
 * rec_out (nullable): device float32 [nt][nrec]; src_adj (nullable): device
 * float32 [nt][nsrc] receives F^T of the residual.  workspace: device, at
 * least fd_gradient_workspace_bytes for the same (nt, nrec,
 * checkpoint_every, flags), 256-byte aligned, borrowed for the call's
 * enqueued work.  Errors: FD_ERR_ARG for an unknown flag, a null required
 * pointer, a 16-bit grid or 16-bit p codes (FD_PARAM_Q16); FD_ERR_NOMEM for
 * a short workspace; otherwise as for fd_forward.
 */
int fd_gradient(fd_grid *grid, const fd_shot *shot, int nt, double dt,
                const float *d_obs_dev, int checkpoint_every, int flags,
                void *workspace, size_t ws_bytes,
                double *misfit_dev, double *grad_m_dev, float *rec_out,
                float *src_adj, void *stream);

/* ------------------------------------------------------------------ serving
 * A request loop that admits shots of different grids by an HBM budget,
 * keeps their wavefields resident, and interleaves their steps on the device
 * (continuous batching: a request arriving while others run starts as soon
 * as a slot and memory are free).  The server owns one device arena of
 * hbm_budget_bytes, carved per request.
 */
typedef struct fd_server_desc {
    int device;                /* HIP device ordinal */
    size_t hbm_budget_bytes;   /* arena size; admission never exceeds it */
    int max_slots;             /* requests resident at once, >= 1 */
    int steps_per_round;       /* steps enqueued per request per scheduler round, 0 selects 50 */
    int policy;                /* FD_SERVE_SHARE (0): every resident request gets the next chunk
                                  of steps as soon as its previous one completes (equal shares);
                                  FD_SERVE_SHORTEST (1): preemptive shortest remaining work
                                  first at chunk granularity -- the device holds at most two
                                  chunks, both for the resident request with the fewest
                                  remaining point-steps while it has steps left (a short shot
                                  arriving behind a long one overtakes it at the next chunk
                                  boundary);
                                  FD_SERVE_RATIO (2): as FD_SERVE_SHORTEST, ordered by the
                                  response ratio (age since submission + remaining time) /
                                  remaining time, the remaining time from the device's
                                  measured point-step rate: short shots still go first, and a
                                  long one that has waited is no longer passed */
} fd_server_desc;

#define FD_SERVE_SHARE 0
#define FD_SERVE_SHORTEST 1
#define FD_SERVE_RATIO 2

typedef struct fd_request {
    fd_grid_desc grid;         /* grid of this shot */
    const float *vp_host;      /* host float32 velocity, physical or padded per grid.vp_padded
                                  (copied at submission) */
    int nsrc;
    const double *src_xyz;     /* host [nsrc][ndim] */
    const float *wavelet_host; /* host [nt][nsrc] (copied at submission) */
    int nrec;
    const double *rec_xyz;     /* host [nrec][ndim] */
    int nt;
    double dt;
    float *rec_out_host;       /* host [nt][nrec], written before the ticket completes */
} fd_request;

typedef struct fd_result {
    int status;                /* fd_status of the request */
    double t_submit;           /* seconds on the server's clock */
    double t_start;            /* admission time */
    double t_done;             /* completion time */
    size_t bytes_reserved;     /* arena bytes the request held */
} fd_result;

typedef struct fd_server fd_server;

/* Create a server on desc->device: allocates the arena (one device
 * allocation of hbm_budget_bytes) and max_slots non-blocking streams, and
 * starts one scheduler thread.  FD_ERR_NOMEM if the arena cannot be had. */
int fd_server_create(const fd_server_desc *desc, fd_server **out);
/* Copy the request's host inputs and queue it; returns at once.  A request
 * larger than the whole budget completes with FD_ERR_NOMEM (at fd_wait). */
int fd_submit(fd_server *srv, const fd_request *req, uint64_t *ticket);
/* Block until the ticket completes or timeout_s passes (FD_ERR_TIMEOUT);
 * timeout_s < 0 waits forever.  A completed ticket is collected once: a
 * second wait, or a wait on a ticket never issued, returns FD_ERR_ARG (a
 * concurrent waiter that loses the race gets FD_ERR_STATE).  A failed
 * request returns its status with the worker's message in fd_last_error. */
int fd_wait(fd_server *srv, uint64_t ticket, double timeout_s, fd_result *result);
/* Bytes of the request's reservation (what admission charges against the budget). */
int fd_request_bytes(const fd_request *req, size_t *bytes);
/* Server-wide counters: peak arena bytes in use and peak resident requests. */
int fd_server_stats(fd_server *srv, size_t *peak_bytes, int *peak_slots);
/* Finish all queued work, then release the arena. */
int fd_server_destroy(fd_server *srv);

/* ---------------------------------------------------------------- diffusion
 * The problem the thesis benchmarks (Section 5.1.2): u_t = nu (u_xx + u_yy)
 * on a 2D grid, first order in time,
 *   u^{n+1} = u^n + nu dt Lap_h u^n,
 * with the same space-order-so weights and zero extension as above.  The
 * so-2 case is the printed kernel of Sections 3.2.2 and 5.1.5.
 */
typedef struct fd_diffusion_desc {
    int shape[2];          /* points (x, y), each >= 2 */
    double spacing[2];     /* h_x, h_y > 0 */
    int space_order;       /* even, 2..16 */
    double nu;             /* diffusivity > 0 */
    int time_block;        /* steps per launch: 0 = automatic (8 at so 2 and 4,
                              4 at so 8, where the LDS-blocked kernel beats one
                              step per launch, else 1), 1 = one step per launch,
                              k > 1 = at most min(k, 16 / (so/2)) */
} fd_diffusion_desc;

/* Device workspace for fd_diffusion_run (two pitched float32 fields). */
int fd_diffusion_workspace_bytes(const fd_diffusion_desc *desc, size_t *bytes);

/* The largest stable time step of the explicit scheme (Section 5.1.2's
 * update u^{n+1} = u^n + nu dt Lap_h u^n): *dt_max = 1 / (2 nu sum_{j odd}
 * c_j sum_a h_a^-2), c_j the maximal-order second-derivative weights of the
 * descriptor's space order; fd_diffusion_run refuses nu dt above nu dt_max.
 * Host only.  FD_ERR_ARG for an invalid descriptor or a null output. */
int fd_diffusion_dt_limit(const fd_diffusion_desc *desc, double *dt_max);

/*
 * nt explicit steps from u0_dev (device float32, dense [Ny][Nx]) into
 * u_out_dev (device float32, dense, may alias u0_dev).  workspace: >= the
 * size above, 256-byte aligned, used during the call only.  FD_ERR_UNSTABLE
 * if nu dt exceeds the explicit limit 1 / (2 sum_{j odd} c_j sum_a h_a^-2).
 * Enqueues on `stream` and returns.
 */
int fd_diffusion_run(const fd_diffusion_desc *desc, void *workspace, size_t ws_bytes,
                     const float *u0_dev, float *u_out_dev, int nt, double dt, void *stream);

/*
 * fd_diffusion_run without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the two fields live in a static device
 * array of 64 MiB inside the library, one per GPU, held until the process
 * ends; nothing is allocated or freed.  Grids whose two pitched fields
 * exceed it (beyond about 2800 x 2800) give FD_ERR_NOMEM.  Every call on a
 * GPU uses that GPU's one array: the call clears it before use, and calls
 * that overlap in time on one GPU (two streams, two threads) race -- order
 * them.  The first call on a device resolves the array's address there.
 * Arguments, result and errors otherwise as fd_diffusion_run.
 */
int fd_diffusion_run_noalloc(const fd_diffusion_desc *desc, const float *u0_dev, float *u_out_dev, int nt,
                             double dt, void *stream);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *fd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FD_H */
