/*
 * fdwave.h - C ABI of the MI355X (gfx950) shaped-stencil acoustic wave library.
 *
 * The library advances the constant-density acoustic wave equation
 *     u_tt - c(x)^2 lap(u) = f                        (Peixoto & Silva, Sec. 3.1, eq. wave_eq)
 * with the explicit leapfrog scheme (Sec. 3.2, eq. time_derivative1) and a
 * symmetric shaped Laplacian stencil (Sec. 3.2, eq. spacexz_derivative2_sym;
 * shapes of Sec. 4.1), an absorbing damping band (Sec. 3.1: eta(x) u_t), a
 * point source and receiver traces (Sec. 5.2).  Per time step n = 0..nt-1:
 *
 *     u^{n+1} = b [ 2 u^n - a u^{n-1} + v (W * u^n) + q s^n delta_{x,xs} ]
 *     trace[n][r] = u^{n+1}(x_r)
 *
 * v = (c dt / h)^2 (squared Courant number, Sec. 3.4.1, eq. courant) is formed
 * once per call in FP64 and rounded to FP32; W * u = sum_d w_d u(x + d) with
 * u = 0 beyond the shot window; q = dt^2 / h^ndim; a = 1 - eta dt / 2,
 * b = 1 / (1 + eta dt / 2), eta = eta_max * sum_axes (depth_into_band / nb)^2.
 * The stencil is evaluated in the centre-free difference form
 * sum_{d != 0} w_d (u(x + d) - u(x)), which equals W * u whenever the weights
 * satisfy the zero-sum (r = 0) condition of Sec. 3.3.1, eq. taylor_system_r0;
 * fd_weights_set enforces that condition.  The time stepping carries the
 * state (u^n, d^n), d^n = u^n - u^{n-1}, and advances it exactly as
 *     d^{n+1} = [(1 - e) d^n + v (W * u^n) + q s^n delta_{x,xs}] / (1 + e),
 *     u^{n+1} = u^n + d^{n+1},   e = eta dt / 2
 * (the update above, rearranged), so that the per-step change is stored at
 * full FP32 precision; initial and final states, and checkpoints, are given
 * in that form.
 *
 * Conventions for every entry point:
 *  - Arrays are row-major with x fastest: 2D [nz][nx], 3D [nz][ny][nx].
 *    Coordinates are given x first: (x, z) in 2D, (x, y, z) in 3D.
 *  - [dev] marks a pointer to device memory on the current HIP device.  All
 *    such memory is allocated and owned by the caller; the library never frees
 *    it.  [host] marks host memory, read during the call only.
 *  - Every function returns an fd_status.  Arguments are validated before any
 *    work is queued; on error nothing is queued and fd_last_error() returns a
 *    message.  No C++ exception crosses this interface and nothing is printed.
 *  - Device work is queued asynchronously on `hip_stream` (a hipStream_t, or
 *    NULL for the null stream) unless a flag below asks for a synchronising
 *    check.  Caller buffers must stay valid until that work has finished.
 *  - The library keeps only host-side state: the registered stencils and a
 *    cache of instantiated HIP graphs.  Scratch memory is the caller's
 *    `workspace` (size from fd_workspace_bytes, 256-byte aligned).
 */
#ifndef FDWAVE_H
#define FDWAVE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FD_OK = 0,
    FD_EINVAL = 1,        /* invalid argument (sizes, indices, pointers) */
    FD_EUNSTABLE = 2,     /* weights or time step violate the stability limit */
    FD_ENOMEM = 3,        /* workspace too small */
    FD_EDEVICE = 4,       /* a HIP runtime call failed */
    FD_ENONFINITE = 5,    /* non-finite values found (check_finite) */
    FD_EUNSUPPORTED = 6   /* valid request with no compiled kernel (shape, radius, tile) */
} fd_status;

typedef enum {
    FD_CROSS = 0,    /* |d_i| <= M on one axis only (Sec. 4.1, P = Q = 0) */
    FD_RHOMBUS = 1,  /* sum |d_i| <= M (Sec. 4.1: Q = floor(M/2), P0(q) = q,
                        P(q) = M - q); in 3D the L1 ball */
    FD_SQUARE = 2,   /* max |d_i| <= M (Sec. 4.1: Q = M, P0(q) = q, P(q) = M) */
    FD_CROSS_RHOMBUS = 3,  /* 2D: the cross of radius M plus the rhombus
                              |x| + |z| <= N, 0 <= N <= M (Sec. 4.1:
                              Q = floor(N/2), P0(q) = q, P(q) = N - q) */
    FD_CROSS_SQUARE = 4    /* 2D: max(|x|, |z|) <= M and min(|x|, |z|) <= N,
                              0 <= N <= M, a cross with arms N cells thick
                              (Sec. 4.1: Q = N, P0(q) = q, P(q) = M) */
} fd_shape;

#define FD_MAX_RADIUS 8      /* largest M with compiled kernels */
#define FD_MAX_ORBITS 64     /* largest number of unique weights per stencil */
#define FD_MAX_STENCILS 256  /* registered stencils per process */

/*
 * Unique-weight structure of a stencil (Sec. 4.1, Fig. stencils: one weight
 * per orbit of the axis-permutation / sign-flip symmetry, Sec. 3.2).
 * An orbit is named by its representative, the absolute offsets sorted in
 * descending order; orbits are listed in ascending lexicographic order of
 * the representative, so orbit 0 is the centre.
 *   ndim     2 or 3;  shape an fd_shape;  M the radius, 1..FD_MAX_RADIUS
 *   reps     [host, out, may be NULL] nw*ndim representatives
 *   counts   [host, out, may be NULL] nw point counts per orbit
 *   nw       [host, out] number of orbits
 * Errors: FD_EINVAL for bad ndim/shape/M or nw == NULL.
 */
int fd_orbits(int ndim, int shape, int M, int* reps, int* counts, int* nw);

/*
 * fd_orbits for shapes with an inner size N (FD_CROSS_RHOMBUS,
 * FD_CROSS_SQUARE: 2D only, 0 <= N <= M); the basic shapes take N = 0, and
 * fd_orbits(...) is fd_orbits_n(..., N = 0, ...).  Errors: FD_EINVAL for a bad
 * combination of ndim, shape, M and N.
 */
int fd_orbits_n(int ndim, int shape, int M, int N, int* reps, int* counts, int* nw);

/*
 * Register a stencil: one FP64 weight per orbit, in fd_orbits order, scaled
 * so that h^2 lap(u)(x) ~ sum_d w_d u(x + d) (Sec. 3.2).  Checks
 *   - nw matches fd_orbits (else FD_EINVAL);
 *   - the zero-sum condition |sum_o count_o w_o| <= 1e-9 sum_o count_o |w_o|
 *     (Sec. 3.3.1, eq. taylor_system_r0; else FD_EINVAL);
 *   - the symbol S(k) = sum_d w_d cos(k.d) is <= 0 on a dense sample of the
 *     Brillouin zone [0, pi]^ndim (else FD_EUNSTABLE: the scheme is unstable
 *     for every time step, Sec. 3.4.1, eq. full_disp).
 * Stores the FP32-rounded weights and the FP64 stability limit
 * C_lim = 2 / sqrt(max_k -S(k)) (largest Courant number with |cos(w dt)| <= 1).
 *   w           [host] nw weights
 *   stencil_id  [host, out] handle for fd_shot.stencil_id
 * Thread-safe.  Registering identical weights again returns the same id.
 */
int fd_weights_set(int ndim, int shape, int M, const double* w, int nw, int* stencil_id);

/*
 * fd_weights_set for shapes with an inner size N (see fd_orbits_n); weights in
 * fd_orbits_n order.  Same checks, errors and handle.  N-shapes without
 * off-axis points (cross-rhombus N <= 1, cross-square N = 0) run the cross
 * kernels; the others run the dense 2D kernels.
 */
int fd_weights_set_n(int ndim, int shape, int M, int N, const double* w, int nw, int* stencil_id);

/* FP64 stability limit of a registered stencil ([host, out] c_lim). */
int fd_cfl_limit(int stencil_id, double* c_lim);

/* The grid, time axis and damping band shared by all shots of a call. */
typedef struct {
    int ndim;              /* 2 or 3 */
    int nt;                /* time steps, >= 1 */
    long long n[3];        /* model extent along x, y, z; n[1] = 1 in 2D */
    double h;              /* grid spacing (m), > 0 */
    double dt;             /* time step (s), > 0 */
    int nb;                /* damping band width in cells (0: no damping) */
    double eta_max;        /* peak damping (1/s) at the outer edge of the band, >= 0 */
    double vmax;           /* maximum velocity used for the stability check */
    int check_finite;      /* 1: synchronise at the end and return FD_ENONFINITE
                              if traces hold NaN/Inf, FD_EINVAL if a receiver
                              coordinate lay outside its window or a velocity
                              was not positive and finite, FD_EUNSTABLE if a
                              velocity c of the model has c dt / h above the
                              smallest C_lim of the call's stencils (vmax
                              understated: the run may have blown up) */
    int flags;             /* FD_NO_GRAPH | FD_NO_BATCH, 0 for the default path */
} fd_grid;

/* fd_grid.flags: the plain execution forms, kept as baselines (results are
 * identical across forms; any other bit is rejected with FD_EINVAL).
 * FD_NO_GRAPH: queue every kernel launch directly instead of replaying a
 *              cached HIP graph of the whole call.
 * FD_NO_BATCH: run the shots of a multi-shot call one after the other with
 *              the single-shot kernels instead of batched launches on
 *              concurrent branches. */
#define FD_NO_GRAPH 1
#define FD_NO_BATCH 2

/* One shot: a window into the model, its stencil, source and receivers. */
typedef struct {
    long long origin[3];     /* window origin in the model (x, y, z) */
    long long extent[3];     /* window extent (x, y, z); y = 1 in 2D */
    int stencil_id;          /* from fd_weights_set, same ndim as the grid */
    int src[3];              /* source node, window coordinates (x, y, z) */
    const float* wavelet;    /* [dev] nt samples s(n dt) of the source (unscaled) */
    int nrec;                /* number of receivers, >= 0 */
    const int* rec;          /* [dev] nrec*ndim window coordinates, x first.
                                Coordinates outside the window are skipped
                                (their traces are 0) and flagged (check_finite) */
    float* traces;           /* [dev, out] nt*nrec: traces[n*nrec + r] = u^{n+1}(rec r) */
    const float* trace_adj;  /* [dev] fd_adjoint_gradient only: dJ/dtraces, nt*nrec */
    const float* init_diff;  /* [dev, optional] d^0 = u^0 - u^{-1} over the window (NULL: zeros) */
    const float* init_cur;   /* [dev, optional] u^0 over the window (NULL: zeros) */
    float* final_diff;       /* [dev, optional out] d^{nt} = u^{nt} - u^{nt-1} over the window
                                (with final_cur: the state a later call resumes from,
                                bitwise, as init_diff / init_cur) */
    float* final_cur;        /* [dev, optional out] u^{nt} over the window */
    float* ckpt;             /* [dev, optional] forward checkpoints: with
                                ckpt_every = K > 0, ceil(nt/K) pairs of window
                                fields; pair j (at ckpt + 2 j npts, npts = window
                                points) holds the state (d^{jK}, u^{jK}).  Written
                                by fd_forward, read by fd_adjoint_gradient (which
                                then skips its own forward pass) */
} fd_shot;

/*
 * Forward modelling of nshots shots over one velocity model.
 *   vel        [dev] model-sized velocity c (m/s), all > 0
 *   shots      [host] nshots descriptors; windows must lie inside the model
 *   nshots     >= 1.  nshots == 1 runs one kernel launch per time step.
 *              nshots > 1 in 2D: the
 *              shots are grouped by stencil variant (shape, M) and each time
 *              step is one launch per group over the tiles of all its shots
 *              (ragged windows allowed); the groups run concurrently on up to
 *              four graph branches; batched tiles are fixed (8 rows per
 *              thread for the forward steps of dense shapes, 4 otherwise).
 *              nshots > 1 in 3D: the shots run concurrently on up to four
 *              branches with the single-shot kernels
 *   ckpt_every 0, or K in [1, nt]: every shot whose ckpt is set receives the
 *              checkpoints (d^{jK}, u^{jK}), j = 0 .. ceil(nt/K) - 1, that
 *              fd_adjoint_gradient with the same K consumes (the states an
 *              FWI gradient needs from the forward pass, Sec. 7).  A shot with
 *              ckpt set and K = 0 is FD_EINVAL
 *   workspace  [dev] >= fd_workspace_bytes(g, shots, nshots, 0, 0) bytes
 *   hip_stream hipStream_t to queue on
 * Stability: vmax * dt / h must not exceed the stencil's C_lim (FD_EUNSTABLE,
 * checked before any work is queued); the velocities themselves are checked
 * against C_lim on the device and reported with check_finite.
 * The time loop is replayed from a cached HIP graph when the same arguments
 * are seen again.
 */
int fd_forward(const fd_grid* g, const float* vel, const fd_shot* shots, int nshots, int ckpt_every,
               void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * fd_forward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): one
 * shot, no checkpoints, its scratch (flags, v, the shot's fields and
 * receiver indices) in a fixed array of FD_NOALLOC_SCRATCH_BYTES that the
 * library keeps in device memory on each GPU it runs on until the process
 * ends.  The caller still passes the inputs and outputs (vel, shot).  Kernel
 * launches go directly onto hip_stream (no graphs, no library streams); the
 * call makes no device or pinned-host allocation.  Results are those of
 * fd_forward (same kernels).
 *   shot      [host] one shot; ckpt must be NULL (FD_EINVAL otherwise)
 * Errors: FD_ENOMEM when the call needs more scratch than the array holds
 * (4 B per model point for v plus 12 B per window point for the fields, plus
 * 8 B per receiver); otherwise those of fd_forward.  Every call on a GPU
 * uses that GPU's one array: calls that overlap in time on one GPU (two
 * streams, two threads) race and must be serialised by the caller.  The
 * array keeps the last call's contents; a call initialises everything it
 * reads.
 */
#define FD_NOALLOC_SCRATCH_BYTES (64ull << 20)
int fd_forward_noalloc(const fd_grid* g, const float* vel, const fd_shot* shot, void* hip_stream);

/*
 * Exact discrete adjoint of fd_forward and the gradient dJ/dc of a scalar
 * misfit J(traces), given trace_adj = dJ/dtraces for each shot.  The adjoint
 * field psi runs backwards in time with the forward operator (W is symmetric),
 *     psi^k = b [ 2 psi^{k+1} - a psi^{k+2} + v (W * psi^{k+1}) + v rho^{k-1} @ x_r ],
 * k = nt..1, psi^{nt+1} = psi^{nt+2} = 0, and
 *     dJ/dc(x) += sum_{k=1..nt} (2 / c(x)) psi^k(x) (W * u^{k-1})(x).
 * The forward field is rebuilt from checkpoints of the state (d^k, u^k) taken
 * every ckpt_every steps and recomputed one segment at a time into the
 * workspace.
 * The paper points to this use of its stencils for FWI gradients (Sec. 7);
 * the adjoint recursion is the exact discrete adjoint of the forward scheme.
 *   grad        [dev, in/out] model-sized; the gradient of every shot is ADDED
 *   ckpt_every  segment length K, 1 <= K <= nt
 *   shots[i].ckpt  NULL: the call runs the forward pass itself (taking the
 *               checkpoints into the workspace) and rewrites the traces;
 *               set: the checkpoints an fd_forward with the same K, grid,
 *               velocity and shot wrote there; the forward pass is skipped
 *               and the traces are left alone.  In a multi-shot 2D call
 *               either every shot or none sets ckpt (FD_EINVAL otherwise)
 * Other arguments as in fd_forward.
 */
int fd_adjoint_gradient(const fd_grid* g, const float* vel, const fd_shot* shots, int nshots,
                        int ckpt_every, float* grad, void* workspace, size_t ws_bytes,
                        void* hip_stream);

/*
 * Workspace size in bytes for fd_forward (mode 0) or fd_adjoint_gradient
 * (mode 1, with segment length ckpt_every; shots that pass saved checkpoints
 * need no checkpoint storage in it).  Returns 0 for invalid input.
 */
size_t fd_workspace_bytes(const fd_grid* g, const fd_shot* shots, int nshots, int mode,
                          int ckpt_every);

/*
 * Adjoint options: checkpointing scheme and gradient parameter.
 *
 * FD_CKPT_SEGMENT: the state (d^{jK}, u^{jK}) stored every K = ckpt_every
 *   steps, each segment recomputed into K + 1 fields (2 ceil(nt/K) + K + 1
 *   window fields per shot, one extra forward pass; none of the 2 ceil(nt/K)
 *   when the shots bring saved checkpoints); multi-shot 2D calls run batched.
 * FD_CKPT_REVOLVE: binomial checkpointing with nsnap snapshots of the state
 *   (d^k, u^k) (Griewank & Walther, ACM TOMS 26, 2000, Algorithm 799):
 *   2 nsnap + 6 window fields, and the least number of forward steps any
 *   schedule with nsnap snapshots needs (fd_revolve_plan gives it).  For
 *   large grids whose segment storage does not fit (3D FWI).  The shots of
 *   a call run one after another with the single-shot kernels; saved
 *   checkpoints (fd_shot.ckpt) are FD_EINVAL with this scheme.
 *
 * The gradient is dJ/dc (FD_PARAM_VELOCITY), dJ/ds for the slowness s = 1/c
 * (FD_PARAM_SLOWNESS: -c^2 dJ/dc) or dJ/dm for m = 1/c^2 (FD_PARAM_M:
 * -(c^3/2) dJ/dc); the factor is applied per term inside the adjoint
 * kernels.  Results are identical across checkpointing schemes (the
 * recomputed forward states are bitwise those of the first pass).
 */
#define FD_CKPT_SEGMENT 0
#define FD_CKPT_REVOLVE 1
#define FD_PARAM_VELOCITY 0
#define FD_PARAM_SLOWNESS 1
#define FD_PARAM_M 2

typedef struct {
    int ckpt;         /* FD_CKPT_SEGMENT or FD_CKPT_REVOLVE */
    int ckpt_every;   /* FD_CKPT_SEGMENT: segment length K, 1 <= K <= nt */
    int nsnap;        /* FD_CKPT_REVOLVE: snapshots, 0 <= nsnap <= nt */
    int param;        /* FD_PARAM_VELOCITY, FD_PARAM_SLOWNESS or FD_PARAM_M */
} fd_adjoint_opts;

/* fd_adjoint_gradient with options (opts [host], required); grad receives
 * the gradient of the chosen parameter (ADDED).  FD_EINVAL for unknown
 * values in opts. */
int fd_adjoint_gradient_ex(const fd_grid* g, const float* vel, const fd_shot* shots, int nshots,
                           const fd_adjoint_opts* opts, float* grad, void* workspace, size_t ws_bytes,
                           void* hip_stream);

/* Workspace bytes of fd_adjoint_gradient_ex (0 for invalid input). */
size_t fd_adjoint_workspace_bytes(const fd_grid* g, const fd_shot* shots, int nshots,
                                  const fd_adjoint_opts* opts);

/*
 * The binomial plan that FD_CKPT_REVOLVE executes for nt steps and nsnap
 * snapshots, as (op, arg) pairs in order:
 *   FD_OP_ADVANCE  t   advance the current state to S_t = (u^{t-1}, u^t)
 *   FD_OP_STORE    j   copy the current state into snapshot j (0 <= j < nsnap)
 *   FD_OP_RESTORE  j   make snapshot j current (j = -1: the initial state S_0)
 *   FD_OP_ADJOINT  k   adjoint iteration k on the current state S_k
 * ADJOINT ops appear for k = nt .. 1 in that order.
 *   ops        [host, out, optional] 2 * max_ops ints
 *   nops       [host, out] number of ops (even when ops is NULL or too short)
 *   fwd_steps  [host, out, optional] forward steps of the plan (each ADVANCE
 *              from the current state's step to t counts t minus that step)
 * FD_EINVAL for nt < 1, nsnap < 0 or nsnap > nt; FD_ENOMEM (with *nops set)
 * when max_ops is smaller than the plan.
 */
#define FD_OP_ADVANCE 0
#define FD_OP_STORE 1
#define FD_OP_RESTORE 2
#define FD_OP_ADJOINT 3
int fd_revolve_plan(int nt, int nsnap, int* ops, long long max_ops, long long* nops, long long* fwd_steps);

/*
 * Kernel tile configuration used for a stencil: rows per thread along the
 * marching axis (2D: z; 3D: y) and the z-chunk of the 3D kernels.
 * fd_set_tile overrides the built-in choice (as found by the autotuner);
 * rows must be one of 1, 2, 4, 8 and zchunk a multiple of 8 in [8, 4096].
 * The setting applies to single-shot kernels (and to shots run one after the
 * other with FD_NO_BATCH); batched 2D calls take their forward tiles from
 * fd_set_batch_tile and run their adjoint steps at 4 rows.  The results do
 * not depend on the tile configuration.
 */
int fd_set_tile(int stencil_id, int rows, int zchunk);
int fd_get_tile(int stencil_id, int* rows, int* zchunk);

/*
 * Tile of a 2D stencil's variant group in the forward steps of batched
 * calls (nshots > 1): rows per thread, 4 (64 x 16 tiles) or 8 (64 x 32, not
 * for crosses), or 0 for the built-in choice (8 for dense shapes, 4 for
 * crosses).  The groups of a batched call run concurrently, so the best tile
 * differs from the single-shot one; the autotuner times whole batched calls
 * to choose it.  Results do not depend on the setting.  fd_get_batch_tile
 * returns the rows in effect.
 * Errors: FD_EINVAL (unknown stencil, rows not 0, 4 or 8), FD_EUNSUPPORTED
 * (3D stencil; rows = 8 for a cross).
 */
int fd_set_batch_tile(int stencil_id, int rows);
int fd_get_batch_tile(int stencil_id, int* rows);

/*
 * Time steps per kernel launch of the forward (kept for callers of the
 * interface): every kernel advances one step per launch, so 1 is the only
 * value; 2 returns FD_EUNSUPPORTED, anything else FD_EINVAL.
 */
int fd_set_time_block(int stencil_id, int steps);
int fd_get_time_block(int stencil_id, int* steps);

/* Message for the last non-OK return on this thread ("" if none). */
const char* fd_last_error(void);

/*
 * Dispersion metrics of Appendix A between numerical and reference traces
 * (e.g. a coarse run and a fine-grid or analytic reference at the same
 * receivers), per receiver:
 *   gamma^F_k = (wrap(phi(A_k) - phi(A'_k)) / pi) |A_k| / max_k |A_k|,
 *     A_k = sum_n u_n exp(-2 pi i k n / nt), k = 0..nt-1 (eq. gammadft);
 *   ||gamma^F||_2 = sqrt(1/nt sum_k gamma_k^2) (eq. norm2gammastdft);
 *   ||gamma^W||_2 of the Morlet CWT measure (eqs. cwt1-cwt3, gammacwt,
 *     norm2gammastcwt) over nscale scales, one per DFT frequency
 *     f_j = j / (nt dt), j = 1..nscale, s_j = (w0 + sqrt(2 + w0^2)) / (4 pi f_j).
 * Amplitudes are sqrt(Re^2 + Im^2); phases atan2(Im, Re) in (-pi, pi]; the
 * phase difference is moved into (-pi, pi] by +-2 pi.  Transforms in FP64.
 *   num, ref    [dev] traces: row n (time) of num starts at num + n*ld_num and
 *               holds nrec receivers (ld_num = nrec for the fd_shot.traces
 *               layout; a larger stride reads every k-th row of a finer
 *               run's traces in place); likewise ref with ld_ref (>= nrec)
 *   dt          sample interval (s); used by the CWT
 *   nscale      number of CWT scales (0: no CWT), <= nt/2
 *   omega0      Morlet centre frequency (the usual choice is 6)
 *   gamma_dft   [dev, out, may be NULL] nrec*nt: gamma^F of receiver r at r*nt + k
 *   norm_dft    [dev, out] nrec per-receiver ||gamma^F||_2
 *   norm_cwt    [dev, out, may be NULL] nrec per-receiver ||gamma^W||_2
 *   workspace   [dev] >= fd_dispersion_workspace_bytes(nt, nrec, norm_cwt ? nscale : 0),
 *               256-byte aligned
 * A receiver whose numerical trace is identically zero (max |A| = 0, where
 * eq. gammadft divides 0 by 0) gets gamma = 0 at every bin and both norms 0:
 * the amplitude weight of a trace without energy is read as 0.
 * The average and maximum over receivers (eqs. norm2gammarecdftavg ..
 * norm2gammareccwtmax) are reductions of norm_dft / norm_cwt by the caller.
 * FFTs run in rocFFT; its plans (and any work buffer they need) are cached
 * by the library per device, length and batch until the process ends.
 * Asynchronous on hip_stream.  Errors: FD_EINVAL, FD_ENOMEM, FD_EDEVICE.
 */
size_t fd_dispersion_workspace_bytes(int nt, int nrec, int nscale);
int fd_dispersion(const float* num, long long ld_num, const float* ref, long long ld_ref, int nt, int nrec,
                  double dt, int nscale, double omega0, float* gamma_dft, double* norm_dft, double* norm_cwt,
                  void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * Error norms of Sec. 6.1.1 between a numerical solution and a reference
 * read through strides (e.g. a run on a grid refined r times, sampled on the
 * coarse nodes and times without a copy):
 *   e(i, j, k) = num[i sn[0] + j sn[1] + k sn[2]] - ref[i sr[0] + j sr[1] + k sr[2]]
 * over the box 0 <= i < n[0], 0 <= j < n[1], 0 <= k < n[2] (element strides,
 * any sign; unused axes have extent 1).
 *   num, ref    [dev] float32
 *   num_stride, ref_stride, n  [host] 3 values each
 *   out         [dev, out] 3 doubles: sum |e|, sum e^2, max |e| (FP64
 *               accumulation, a fixed reduction order: repeatable); the
 *               paper's L1 = out[0] / h^2, L2 = sqrt(out[1]) / h, Linf = out[2]
 *               (tau for h on traces) are the caller's
 *   workspace   [dev] >= FD_ERROR_NORMS_WS_BYTES bytes, 256-byte aligned
 * Asynchronous on hip_stream.  Errors: FD_EINVAL, FD_ENOMEM, FD_EDEVICE.
 */
#define FD_ERROR_NORMS_WS_BYTES 24576
int fd_error_norms(const float* num, const long long* num_stride, const float* ref, const long long* ref_stride,
                   const long long* n, double* out, void* workspace, size_t ws_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FDWAVE_H */
