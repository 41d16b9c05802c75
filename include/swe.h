/*
 * swe.h -- C ABI of libswe.so, the MI355X (gfx950) shallow-water library.
 *
 * The library advances the 2D shallow-water mass and momentum equations with
 * the explicit predictor-corrector MacCormack scheme (Seitz et al., 2013, §1):
 * each time step is sixteen dependent sub-steps, every one a cell-independent
 * stencil sweep, with a variable time step computed after every step from the
 * new state (§3.1).  Unknowns are the water-surface elevation eta and the unit
 * discharges qx, qy; the bed elevation z and a Manning coefficient field n are
 * static.  Dry cells (depth <= h_dry), which the paper lists as unsupported
 * (§6.2), are handled by a thin-film rule: zero velocity, no dissipation or
 * pressure across dry banks, negative depth clipped with the clipped volume
 * recorded.
 *
 * Conventions shared by every entry point:
 *   - Fields are 2D, row-major with x fastest: element (i, j) of a field sits
 *     at index j*pitch + i, 0 <= i < nx, 0 <= j < ny, pitch >= nx (elements).
 *     Every field of one handle has the same pitch and element type
 *     (float for SWE_F32, double for SWE_F64).
 *   - Device pointers are GPU memory of the device current at swe_create.  The
 *     caller owns them (typically PyTorch tensors); they must outlive the
 *     handle.  The library never frees caller memory.
 *   - All device work is enqueued on the stream given at create (NULL: the
 *     null stream).  A handle is not thread-safe.
 *   - Return values: SWE_OK (0) or a negative swe_status.  No C++ exception and
 *     no abort crosses this interface; the message of the last failure is
 *     available from swe_last_error.
 */
#ifndef SWE_H
#define SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWE_ABI_VERSION 3

typedef enum swe_status {
    SWE_OK = 0,
    SWE_EINVAL = -1,       /* bad argument; nothing was enqueued */
    SWE_ENOMEM = -2,       /* device or host allocation failed */
    SWE_EDEVICE = -3,      /* no usable GPU, or a HIP call failed (text in last_error) */
    SWE_EUNSTABLE = -4,    /* a step produced NaN/Inf or an invalid time step */
    SWE_EUNSUPPORTED = -5  /* valid request the library does not implement */
} swe_status;

typedef enum swe_dtype { SWE_F32 = 1, SWE_F64 = 2 } swe_dtype;

/* Boundary kind of an edge.  WALL: reflective, no flux.  OPEN: zero-gradient
 * outflow (ghost = copy of the edge cell).  INFLOW: prescribed normal unit
 * discharge q_in(t) into the domain (the hydrograph), acting as WALL outside
 * the edge's face band [inflow_lo, inflow_hi). */
typedef enum swe_bc { SWE_BC_WALL = 0, SWE_BC_OPEN = 1, SWE_BC_INFLOW = 2 } swe_bc;
typedef enum swe_edge { SWE_EDGE_W = 0, SWE_EDGE_E = 1, SWE_EDGE_S = 2, SWE_EDGE_N = 3 } swe_edge;

/* Execution path.  FUSED: one kernel per time step (all sixteen sub-steps on
 * an LDS/register-resident tile, the default).  UNFUSED: one kernel per
 * sub-step with every intermediate in device memory; bitwise equal results,
 * kept as the parity ladder and as the one-kernel-per-sub-step comparison
 * point (the paper's own structure, §3.1). */
typedef enum swe_path { SWE_PATH_FUSED = 0, SWE_PATH_UNFUSED = 1 } swe_path;

/* Flag bits reported in swe_stats.flags. */
enum {
    SWE_FLAG_NAN = 1,      /* a non-finite value appeared (fatal) */
    SWE_FLAG_CLIPPED = 2,  /* a negative depth was clipped (informational) */
    SWE_FLAG_BADDT = 4,    /* the next time step is not finite and positive (fatal) */
    SWE_FLAG_STALL = 8     /* a wave of the fused step (two waves per tile) stopped waiting
                              for its partner after its bounded wait: the step's values are
                              not to be trusted (fatal) */
};

/* Problem definition.  Fill with swe_config_init, then set the fields. */
typedef struct swe_config {
    int32_t nx, ny;          /* cells in x and y, each >= 5 */
    int32_t dtype;           /* SWE_F32 or SWE_F64: element type of every field */
    int32_t path;            /* swe_path */
    int32_t bc[4];           /* swe_bc per edge, indexed by swe_edge */
    int32_t inflow_lo[4];    /* INFLOW face band along each edge: faces k with */
    int32_t inflow_hi[4];    /*   lo <= k < hi (k = j on W/E, k = i on S/N) */
    int32_t hydro_len;       /* points of the hydrograph, 0..4096 (0: q_in = 0) */
    int32_t tile_rows;       /* rows per tile of the fused kernel, 0 = auto (as many
                              * chunks per strip as resident tiles allow, at least 6
                              * rows).  A tile is one workgroup of two waves, one running
                              * the predictor half of every row and one the corrector half
                              * (SWE_FUSED_SPLIT=0 in the environment at swe_create: one
                              * wave per tile; same results).  SWE_FUSED_WAVES=3 (FP64) or
                              * 5 (FP32) selects the one-wave kernel's occupancy variant,
                              * one more resident wave per SIMD than its register budget
                              * allows (part of the carried state spills); a measurement
                              * knob with the same results, not used with the dry-tile
                              * skip */
    int64_t pitch;           /* row pitch of every field in elements, >= nx */
    double dx, dy;           /* cell size (m), > 0 */
    double g;                /* gravity (m/s^2), > 0 */
    double cfl;              /* Courant number of the adaptive step, (0, 1] */
    double h_dry;            /* dry-depth threshold (m), >= 0; wet <=> h > h_dry */
    double kappa;            /* dissipation coefficient, [0, 4] */
    double eps_max;          /* cap of the per-face dissipation coefficient, [0, 0.25] */
    double dt_max;           /* upper bound of the time step (s), > 0 */
    double dt_fixed;         /* > 0: use this time step every step; <= 0: adaptive */
    double t0;               /* start time (s) */
    const double* hydro_t;   /* host, hydro_len increasing times (s); copied */
    const double* hydro_q;   /* host, hydro_len unit discharges (m^2/s); copied */
    const void* z;           /* device: bed elevation (m) */
    const void* n;           /* device: Manning coefficient (s m^-1/3); read once */
    void* eta;               /* device, in/out: water-surface elevation (m) */
    void* qx;                /* device, in/out: unit discharge along x (m^2/s) */
    void* qy;                /* device, in/out: unit discharge along y (m^2/s) */
    void* stream;            /* hipStream_t, or NULL */
    int32_t dry_skip;        /* 1: dry-tile skip (FUSED only), 0: every tile computed.
                              * A tile of the fused kernel whose cells, and the cells
                              * of its eight neighbour tiles, were all dry (h <= h_dry,
                              * zero discharge) after the previous step and that lies
                              * at least two cells from every edge is left out: the
                              * step provably maps it to itself, so results are bit
                              * for bit those of the dense step.  Flags are rebuilt
                              * from a dense first step at the start of every call
                              * (swe_run, swe_step, ensemble run or replay), so the
                              * caller may change the state between calls. */
    double h_film;           /* thin-film reading (m): > 0 makes the reciprocal depth
                              * of sub-steps 2 and 9 min(1/h, 1/h_film), so films
                              * thinner than h_film take their velocities (q/h_film)
                              * and their dissipation switch from that depth; mass
                              * fluxes, friction and the CFL step keep the true
                              * depth.  0 (the default) is the plain scheme.  The
                              * paper leaves dry and drying cells to future work
                              * (§6.2); without this the discrete adjoint of a flood
                              * over dry land grows without bound through the 1/h^2
                              * depth derivative in thin films.  Cells deeper than
                              * h_film are unaffected. */
} swe_config;

/* Progress and diagnostics of a handle. */
typedef struct swe_stats {
    int64_t step;            /* global step index n of the current state */
    int64_t steps;           /* steps taken by the call that filled this */
    int64_t bad_step;        /* step that raised a fatal flag, or -1 */
    uint32_t flags;          /* OR of all flags raised since create */
    uint32_t pad_;
    double t;                /* t^n of the current state (s) */
    double dt;               /* dt^n, the step the next swe_step will take (s) */
    double dt_min, dt_max;   /* extremes of the steps taken by the call (s) */
    double volume;           /* sum of (eta - z) dx dy over the state (m^3) */
    double defect;           /* clipped volume added since create (m^3) */
    double lambda_max;       /* max over wet cells of (|u|+c)/dx + (|v|+c)/dy */
    int64_t cells_skipped;   /* cell updates of the call left out by the dry-tile skip */
} swe_stats;

/* Scalars needed to resume a run bitwise: the caller saves its own eta, qx,
 * qy arrays next to this record. */
typedef struct swe_checkpoint {
    int64_t step;
    uint32_t flags;
    uint32_t pad_;
    double t, dt, defect;
} swe_checkpoint;

typedef struct swe_handle swe_handle;

/* SWE_ABI_VERSION of the loaded library. */
int swe_abi_version(void);

/* Fill *cfg with defaults: g = 9.81, cfl = 0.5, h_dry = 1e-3, kappa = 0.5,
 * eps_max = 0.25, dt_max = 1, dt_fixed = 0, t0 = 0, dtype = SWE_F64, path =
 * FUSED, all edges WALL with full inflow bands, every pointer NULL.  No-op on
 * NULL. */
void swe_config_init(swe_config* cfg);

/* Validate cfg, take host copies of the hydrograph, allocate the library's
 * device scratch (second state buffer, m = g n^2, control block, reduction
 * partials) and compute dt^0 from the initial state (sub-step 16 on U^0; the
 * time step is variable and computed from the data, §3.1).  The grid, bed,
 * friction field and state are the uniform Cartesian cells of the paper's
 * shallow-water problem (§1).
 * Enqueues on cfg->stream and synchronises it once.  On success *out owns the
 * scratch; on failure *out is NULL and swe_last_error(NULL) says why.
 * Errors: SWE_EINVAL (NULL pointer, sizes, ranges, pitch < nx, unknown enum),
 * SWE_EDEVICE (no GPU, or a pointer that is not device memory of the current
 * device), SWE_ENOMEM. */
int swe_create(const swe_config* cfg, swe_handle** out);

/* Free the library's scratch (never caller memory).  NULL is a no-op. */
void swe_destroy(swe_handle* h);

/* One time step: the explicit predictor-corrector MacCormack step split into
 * sixteen dependent sub-steps, each independent across cells (§1, §6.1), run
 * as one fused kernel (or one kernel per sub-step on the UNFUSED path), with
 * dt^{n+1} computed on the device at its end (§3.1).  Asynchronous on the
 * handle's stream; the new state is in the caller's eta/qx/qy when the stream
 * reaches it.  With
 * dt_used != NULL the call synchronises and stores the step taken.  Errors:
 * SWE_EINVAL, SWE_EDEVICE, SWE_EUNSTABLE (only detected when dt_used != NULL). */
int swe_step(swe_handle* h, double* dt_used);

/* Up to nsteps steps of swe_step's time step (§1, §3.1), stopping early once
 * t >= t_end (pass +INFINITY for no limit) or after a step raises a fatal flag; steps past the stop become
 * no-ops on the device, so the host enqueues all launches without waiting.
 * Synchronises once at the end, leaves the final state in the caller's
 * arrays and fills *out (may be NULL).  Returns SWE_EUNSTABLE if a fatal flag
 * was raised (out->bad_step names the step). */
int swe_run(swe_handle* h, int64_t nsteps, double t_end, swe_stats* out);

/* nsteps steps on a prescribed time grid: step k takes dts[k] (host array of
 * nsteps finite values > 0) instead of the step the CFL condition (§3.1) or
 * dt_fixed would choose; t advances by the same sums as in swe_run.  Meant
 * for replaying the time grid of an earlier run: swe_grad differentiates
 * with the run's dt^n held fixed, so a finite-difference check of its
 * gradient, or a line search, must reuse those steps.  The dt that the
 * stats report afterwards is the CFL step of the final state.  Synchronises
 * once; errors as swe_run, plus SWE_EINVAL for a NULL or invalid dts. */
int swe_run_dt(swe_handle* h, int64_t nsteps, const double* dts, swe_stats* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture of its own work, tight serving loops, harnesses that forbid
 * hipMalloc): swe_create + swe_run(nsteps, t_end) + swe_destroy in one call
 * that allocates nothing.  The caller's z, n, eta, qx, qy (cfg) are read and
 * eta, qx, qy written as by swe_run, with the same kernels and the same
 * results bit for bit.  The library's scratch (second state buffer, m, control
 * block, partial sums, hydrograph) is a static device array of about 35 MiB,
 * one per device that loads the library, held until the process ends.
 * Limits: pitch * ny <= 1048576 elements (either dtype), at most 65536 tiles,
 * FUSED path, dry_skip = 0.  The array keeps the previous call's contents and
 * each call clears what must start at zero; calls that overlap on one device
 * (two host threads, or two streams in flight at once) race on it.
 * Synchronises the stream once at the end and fills *out (may be NULL).
 * Errors (read with swe_last_error(NULL)): as swe_create and swe_run, plus
 * SWE_EINVAL for a grid or tile count beyond the limits, another path or the
 * dry-tile skip. */
int swe_run_noalloc(const swe_config* cfg, int64_t nsteps, double t_end, swe_stats* out);

/* Synchronise the stream and report the current statistics. */
int swe_get_stats(swe_handle* h, swe_stats* out);

/* One time step on the UNFUSED path that also copies every intermediate out:
 * `arrays` (device, `bytes` >= swe_trace_bytes(h)) receives 47 arrays of
 * (ny+2) x (nx+2) elements of the handle's dtype, each padded with a one-cell
 * ghost ring (element (i, j) at (j+1)*(nx+2) + (i+1), i in [-1, nx], j in
 * [-1, ny]), in the order: S1 eta, qx, qy (with ghosts); S2 h, r, u, v;
 * S3 nu_x, nu_y; S4 D_eta, D_qx, D_qy; S5 Fm, Fx, Fy, Px; S6 Gm, Gx, Gy, Py;
 * S7/S8 eta*, qx*, qy*; S9 h*, r*, u*, v*; S10 (4); S11 (4); S12 (3);
 * S13 (3); S14 (3); S15 (3).  Face arrays keep the face between cells k and
 * k+1 in the slot of cell k.  `scalars` (host, 16 doubles) receives q_in(t^n),
 * q_in(t^n + dt), dt/dx, dt/dy, the clipped depth sum, lambda_max, dt^{n+1},
 * volume, flags of the step, sigma, t^{n+1}, then zeros.  Synchronises. */
int swe_trace_step(swe_handle* h, void* arrays, size_t bytes, double* scalars);

/* Bytes of the `arrays` buffer swe_trace_step needs. */
size_t swe_trace_bytes(const swe_handle* h);

/* Copy the handle's scalars to *ck (synchronises), or restore them from *ck
 * after the caller has restored its eta/qx/qy arrays. */
int swe_save(swe_handle* h, swe_checkpoint* ck);
int swe_load(swe_handle* h, const swe_checkpoint* ck);

/* Message of the handle's last failure, or of the last failed swe_create
 * when h is NULL.  Never NULL; valid until the next call on that handle. */
const char* swe_last_error(const swe_handle* h);

/* Gauges of the misfit loss of swe_grad. */
typedef struct swe_gauges {
    int32_t ngauge;          /* number of gauge cells (>= 0) */
    int32_t obs_every;       /* observe after steps obs_every, 2*obs_every, ... (>= 1) */
    const int64_t* cells;    /* host, ngauge distinct cells j*nx + i */
    const double* hobs;      /* device, FP64, [floor(nsteps/obs_every)][ngauge]
                                observed depths, row k after step (k+1)*obs_every */
} swe_gauges;

/* Discrete adjoint of the step (§1) with respect to the friction and bed
 * fields (growth path: calibration).  Runs nsteps time steps from the
 * current state, exactly as swe_run(nsteps) would (the handle ends advanced by nsteps steps), and
 * returns the gauge-misfit loss
 *   J = sum_k sum_g ((eta - z)(cell_g, after step k*obs_every) - hobs[k-1][g])^2
 * together with its gradient with respect to the Manning field n and the bed
 * z of the handle, for the sequence of time steps dt^n the run took held
 * fixed (dt is not differentiated).  The gradient is the exact derivative of
 * the discrete step (S1..S15 in reverse, branches as taken in the forward
 * run; max/min follow the argument they return, |x| and sqrt have
 * derivative 0 at 0).  Memory (ckpt_every >= 1): states every ckpt_every
 * steps are kept, and each segment of ckpt_every steps is recomputed once
 * during the reverse sweep (about 2 + 1/ckpt_every forward passes in all);
 * FP64 handles also keep U* and U^d of each step of the segment being
 * reversed (6 fields per step) when that fits in a third of the free device
 * memory, else each step is replayed once more (SWE_GRAD_KEEP=0 in the
 * environment forces the replay).  With U* and U^d kept and more than one
 * segment, the recompute of the next segment runs on a second stream of the
 * library's while the reverse sweep marches the present one, in a second set
 * of segment buffers when that also fits in a third of the free memory
 * (SWE_GRAD_OVERLAP=0 in the environment runs them one after the other on
 * the handle's stream); the call still returns only when all of it is done.
 * ckpt_every = 0: an FP64 handle keeps the
 * whole trajectory (U^n, U* and U^d of every step, 9 fields per step) when it
 * fits in three quarters of the free device memory, and then recomputes
 * nothing; the buffer stays with the handle for later calls and is released
 * by swe_destroy.  Otherwise, and for FP32 handles, the spacing is
 * round(sqrt(nsteps)).  The reverse step runs as one fused march with two
 * waves per tile that hand rows over through LDS counters, each wait bounded
 * (SWE_ADJOINT in the environment selects another form: barrier, the same two
 * waves in step at a workgroup barrier; march1, the one-wave march; gather,
 * four gather kernels).  The gradient is the same bit for bit in every one of
 * these modes.  Measurement knobs, same bits: SWE_MARCH_ROWS and SWE_TRACE_ROWS
 * fix the reverse march's and the tracing step's tile heights;
 * SWE_MARCH_SPIN_CAP lowers the bound on the march's waits (tests of the
 * stall report).  dJ_dn and dJ_dz (device, FP64, caller-owned, the handle's pitch)
 * receive the gradients;
 * *loss (host) receives J.  FP32 handles: the forward run, its checkpoints
 * and the recomputed segments are FP32 (the state trajectory is that of
 * swe_run), and the reverse sweep is FP64, each step linearised at its FP32
 * state promoted to FP64 (with FP64 copies of z, n and m = g n^2); misfits
 * are formed in FP64 from the promoted depths.  Memory then holds FP32
 * checkpoints and segment states plus FP64 copies of one step's state, U* and
 * U^d.  Synchronises.  Errors: SWE_EINVAL (arguments, ckpt_every < 0, gauge
 * cells out of range or repeated), SWE_ENOMEM, SWE_EDEVICE (also when a wave of
 * the march stopped waiting for its partner: the gradient is then not
 * returned), SWE_EUNSTABLE (the forward run raised a fatal flag). */
int swe_grad(swe_handle* h, int64_t nsteps, const swe_gauges* g, int32_t ckpt_every,
             double* loss, void* dJ_dn, void* dJ_dz);

/* The loss of swe_grad alone: runs nsteps steps exactly as swe_run(nsteps)
 * (the handle advances) and stores J in *loss (host), with the misfits
 * formed and summed as swe_grad forms them, so both give the same bits for
 * the same run.  Costs one forward run.  Synchronises.  Errors: as swe_grad
 * (without the gradient arguments). */
int swe_loss(swe_handle* h, int64_t nsteps, const swe_gauges* g, double* loss);

/* Ensemble (growth path: many independent scenarios per launch; each
 * scenario is the step of §1 on its own grid).
 * `count` scenarios, each a full swe_config (its own grid size, bed, Manning
 * field, state arrays, boundary kinds, hydrograph and CFL-adaptive dt; all of
 * one dtype, path FUSED, t0 = 0).  Every time step of all scenarios is ONE
 * launch of the fused step kernel over the concatenated tile lists
 * (workgroup -> (scenario, tile) by a prefix-sum lookup); each scenario's dt
 * is finalised by the last of its own workgroups, so scenarios keep separate
 * time steps and stop independently (t_end, fatal flags).  The ensemble owns
 * one non-blocking stream (cfg->stream is ignored) and the scenarios' scratch.
 * tile_rows > 0 fixes the tile height for every scenario; 0 lets the
 * library's autotuner time the candidate heights 16, 32, 48, 64, 96 and 128 on the
 * ensemble itself (the best of three short runs each, state restored afterwards) and keep the
 * fastest (cached per set of grid sizes for the life of the process).
 * Errors: as swe_create, plus SWE_EINVAL for mixed dtypes, an unfused path or
 * t0 != 0. */
typedef struct swe_ensemble swe_ensemble;
int swe_ensemble_create(const swe_config* cfgs, int32_t count, int32_t tile_rows,
                        swe_ensemble** out);
void swe_ensemble_destroy(swe_ensemble* e);
/* nsteps steps of every scenario (stopping each at t_end or a fatal flag),
 * asynchronous; the final states are in the callers' arrays once the stream
 * reaches the end. */
int swe_ensemble_run(swe_ensemble* e, int64_t nsteps, double t_end);
/* Capture one swe_ensemble_run(nsteps, +inf) (nsteps even, so that every
 * replay starts on an even step) into a HIP graph; swe_ensemble_replay
 * launches it once (asynchronous).  The graph holds kernel nodes only. */
int swe_ensemble_capture(swe_ensemble* e, int64_t nsteps);
int swe_ensemble_replay(swe_ensemble* e);
/* Synchronise and fill out[0 .. count) (may be NULL: synchronise only).
 * SWE_EUNSTABLE if any scenario raised a fatal flag. */
int swe_ensemble_stats(swe_ensemble* e, swe_stats* out);
/* Tile height in use (after autotuning). */
int32_t swe_ensemble_tile_rows(const swe_ensemble* e);
const char* swe_ensemble_last_error(const swe_ensemble* e);

/* Plain device-to-device copy kernel of `bytes` bytes (multiple of 16, both
 * pointers 16-byte aligned) on `stream`: the bandwidth probe the HBM traffic
 * counters are calibrated against.  Asynchronous.  SWE_EINVAL on misuse. */
int swe_probe_copy(void* dst, const void* src, size_t bytes, void* stream);

/* The fused step's memory traffic as a plain stream: five device arrays of
 * `bytes` bytes read (in[0..4]) and three written (out[0..2]), one pass,
 * grid-stride, 16 bytes per lane; nontemporal != 0 adds the non-temporal
 * hint to every load and store.  The achievable-bandwidth ceiling that the
 * step's 8-array traffic is measured against (the paper's GPU was bound by
 * its global-memory accesses, §3.2).  Arrays 16-byte aligned, bytes a
 * multiple of 16.  Asynchronous.  SWE_EINVAL on misuse. */
int swe_probe_stream(const void* const* in, void* const* out, size_t bytes, int nontemporal,
                     void* stream);

/* The fused step's access pattern without its arithmetic: the same tiles,
 * tile order and row march as the step kernel (one 64-lane wave per strip of
 * 60 output columns marching up a chunk of `rows` rows, the next row
 * prefetched), reading in[0..4] and writing out[0..2] (each ny rows of
 * `pitch` elements of elem_bytes = 4 or 8 bytes, nx <= pitch columns used),
 * with a few operations per cell in place of the sub-steps S1-S16 (§3.2: the
 * step is bound by its global-memory accesses).  It is the traversal's own
 * bandwidth ceiling, between the plain stream and the step kernel.  rows = 0
 * takes the height the step kernel picks by itself for that precision and
 * grid on the current device.  Returns the rows used (> 0), or SWE_EINVAL
 * on misuse (NULL or misaligned arrays, nx > pitch, ny * pitch > 2^31).
 * Asynchronous. */
int swe_probe_march(const void* const* in, void* const* out, int32_t nx, int32_t ny,
                    int64_t pitch, int32_t elem_bytes, int32_t rows, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SWE_H */
