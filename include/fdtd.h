/*
 * fdtd.h -- C ABI of the MI355X (gfx950) Yee FDTD library, libfdtd.so.
 *
 * The library advances Maxwell's curl equations on a PEC box cavity with the
 * Yee leapfrog (He, Andersson, Markidis, "Optimizing FDTD Solvers for
 * Electromagnetics: A Compiler-Guided Approach with High-Level Tensor
 * Abstractions", arXiv 2504.09118):
 *   - Sec. 2, Eq. 2: the six component updates; E uses dt/eps, H uses
 *     dt/mu, with the minus sign of Faraday's law as printed in Eq. 2.
 *   - Sec. 2.1, full algorithm listing: each step updates H from the curl
 *     of E, applies the H boundary, updates E from the curl of H, applies the
 *     E boundary.
 *   - Sec. 2.1, naive and slicing curl_Hx listings: forward differences of E
 *     for H, staggered array extents.
 *   - Fig. 1b caption and Sec. 4: PEC walls on a box cavity.
 *
 * Units: the caller chooses them; the library only uses dx, dt and the
 * relative material values. With c = eps0 = mu0 = 1 the coefficients are
 * Ce = dt/(eps_r dx) and Ch = dt/(mu_r dx).
 *
 * Host field layout (all set/get calls): each component is a dense
 * x-fastest array, element (i, j, k) at i + X*(j + Y*k), with extents (X,Y,Z)
 *   Ex (nx, ny+1, nz+1)   Ey (nx+1, ny, nz+1)   Ez (nx+1, ny+1, nz)
 *   Hx (nx+1, ny, nz)     Hy (nx, ny+1, nz)     Hz (nx, ny, nz+1)
 * (in NumPy terms a C-order array of shape (Z, Y, X) indexed [k, j, i]).
 * The order of the six pointers in every array argument is Ex, Ey, Ez, Hx,
 * Hy, Hz. The device layout is private to the library.
 *
 * Time levels (the algorithm listing's H-then-E order): after set_fields,
 * E holds E^0 and H holds H^{-1/2}; after step(n) the state is E^n, H^{n-1/2}.
 *
 * Errors: every call returns an fdtd_status and never throws. On failure
 * fdtd_last_error() returns a thread-local message. A handle whose device
 * work failed enters an error state; later calls on it return FDTD_E_STATE
 * (except fdtd_destroy).
 *
 * Threading: a handle is not thread-safe; different handles may be used from
 * different threads on different streams.
 */
#ifndef FDTD_H
#define FDTD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_solver *fdtd_t;

typedef enum {
    FDTD_OK = 0,
    FDTD_E_ARG = -1,          /* invalid argument (dims, dx, dt, NULL pointer, material value) */
    FDTD_E_CFL = -2,          /* dt violates the Courant limit of the given medium */
    FDTD_E_NOMEM = -3,        /* device memory or the caller's arena is too small */
    FDTD_E_DEVICE = -4,       /* a HIP call or a kernel failed */
    FDTD_E_STATE = -5,        /* NULL / destroyed / errored handle, or fields never set */
    FDTD_E_UNSUPPORTED = -6,  /* option combination not built */
    FDTD_E_TIMEOUT = -7       /* a pool wait ran out of time (nothing failed) */
} fdtd_status;

/*
 * Element types. Host and device buffers passed to set/get calls are FDTD_F64
 * or FDTD_F32. Device field storage may also be 16-bit: FDTD_F16 (IEEE half)
 * or FDTD_BF16 (bfloat16); such fields are widened to FP32 on load, a sweep
 * computes in FP32 (coefficients stay FP32) and rounds to nearest even once
 * when it stores, i.e. once per sweep of tb_steps steps.
 * Compensated storage (FDTD_F16C, FDTD_BF16C) keeps, next to each 16-bit value
 * hi, the rounding residual of the FP32 value x it stands for: q = rint((x -
 * hi) / s) in [-127, 127] as an int8, s = ulp(hi) / 256 (a power of two from
 * hi's exponent). The value is hi + q s, exact in FP32 and within ulp(hi)/512
 * of x, about 2^-20 (FP16) or 2^-17 (BF16) relative per store instead of 2^-11
 * or 2^-8. The three residuals of a node's E (or H) components share one 4-byte
 * record on the device: 2 + 4/3 bytes per value. Built for the temporal kernel.
 */
typedef enum {
    FDTD_F64 = 0,
    FDTD_F32 = 1,
    FDTD_F16 = 2,
    FDTD_BF16 = 3,
    FDTD_F16C = 4,  /* compensated FP16: see below */
    FDTD_BF16C = 5  /* compensated BF16 */
} fdtd_dtype;

/* Field indices in the six-pointer arrays. */
enum { FDTD_EX = 0, FDTD_EY, FDTD_EZ, FDTD_HX, FDTD_HY, FDTD_HZ };

/* Kernel schedules for fdtd_step (all give the same bits for the same storage type). */
typedef enum {
    FDTD_KERNEL_AUTO = 0,      /* the fastest built schedule for the storage type */
    FDTD_KERNEL_PLAIN = 1,     /* two sweeps per step: update H, then update E, in place */
    FDTD_KERNEL_FUSED = 2,     /* one z-marching sweep per step (H then E per plane) */
    FDTD_KERNEL_SLAB = 3,      /* fused sweep with LDS-staged plane tiles */
    FDTD_KERNEL_TEMPORAL = 4   /* tb_steps full steps per sweep (temporal blocking) */
} fdtd_kernel;

/*
 * Per-cell materials, both x-fastest arrays of nx*ny*nz host doubles; NULL
 * means 1 everywhere. The coefficient of an E node (a cell edge) uses the
 * mean eps_r of the four cells sharing the edge, summed as ((a+b)+(c+d))/4;
 * an H node (a face) the mean mu_r of its two cells. The means, divisions and
 * the rounding to the storage type are done in FP64 on the device, once, at
 * fdtd_create. NULL eps_r (mu_r) keeps a single scalar coefficient instead of
 * per-node arrays.
 */
typedef struct {
    const double *eps_r;
    const double *mu_r;
} fdtd_coef;

typedef struct {
    int storage;        /* fdtd_dtype of device fields: FDTD_F32 (default), FDTD_F64, FDTD_F16, FDTD_BF16,
                           FDTD_F16C, FDTD_BF16C (16-bit based storage runs the temporal kernel only) */
    int kernel;         /* fdtd_kernel, default FDTD_KERNEL_AUTO */
    int tb_steps;       /* steps per sweep for FDTD_KERNEL_TEMPORAL, 1..4 (0: library default:
                           4 without per-node Ch, else 3) */
    int device;         /* HIP device ordinal, default 0 */
    void *stream;       /* hipStream_t to enqueue on; NULL: the library creates its own */
    void *arena;        /* caller-owned device memory for all device state; NULL: hipMalloc */
    size_t arena_bytes; /* size of arena in bytes (>= fdtd_required_bytes) */
    double dy, dz;      /* cell size along y and z; 0: dx (cubic cells). Giving either selects
                           rectangular cells (see below) */
} fdtd_opts;

/*
 * Rectangular cells (dx, dy, dz; the naive curl_Hx listing of Sec. 2.1 keeps
 * Dy and Dz): each difference of Eq. 2 is divided by its own spacing. The
 * device stores E_a s_a and H_a s_a with s = (1, dy/dx, dz/dx) (edge
 * integrals in units of dx), in which variables the update is the cubic one
 * with component a's coefficient multiplied by s_a / (s_b s_c) (b, c the other
 * axes); those coefficients are per-node arrays, computed in FP64 like the
 * cubic ones. set/get calls take and return physical values (the scaling is
 * applied in FP64 and rounded once); fdtd_get_coefs and fdtd_diag report the
 * stored variables. Courant limit: dt sqrt(1/dx^2 + 1/dy^2 + 1/dz^2) <
 * sqrt(min eps_r min mu_r). The adjoint and the serving pool take cubic cells.
 */

/* Fill *opts with the defaults listed above. Returns FDTD_E_ARG for NULL. */
int fdtd_opts_default(fdtd_opts *opts);

/*
 * Device bytes fdtd_create needs for these dims, materials and options (the
 * arena size a caller must provide). coef and opts may be NULL (defaults).
 * Returns FDTD_E_ARG for dims < 2 or NULL out.
 */
int fdtd_required_bytes(int nx, int ny, int nz, const fdtd_coef *coef, const fdtd_opts *opts,
                        size_t *out);

/*
 * Create a solver for an nx*ny*nz-cell PEC cavity with cubic cells of size dx
 * and time step dt, and enqueue the coefficient precompute on its stream.
 * Fields start at zero.
 * Checks: nx, ny, nz >= 2; nx*ny*nz <= 2^33; one padded x-y plane
 * (round_up(nx+1, 64) * (ny+1) values, of 8 bytes for FP64 storage and 4
 * bytes otherwise: 16-bit storage sweeps FP32 coefficient planes and 4-byte
 * residual-record planes of the same size) below 2^31 bytes (FDTD_E_ARG);
 * dx, dt finite and > 0; every material value
 * finite and > 0; the Courant limit dt*sqrt(3)/dx < sqrt(min eps_r * min mu_r)
 * (FDTD_E_CFL); a given arena of at least fdtd_required_bytes, and without
 * an arena a need within the byte count in the environment variable
 * FDTD_HBM_BUDGET when it is set (FDTD_E_NOMEM; both checked before any
 * device call, then FDTD_E_NOMEM if hipMalloc fails). Host arrays in coef are
 * read during the call only. The arena, if given, is borrowed until
 * fdtd_destroy and must stay allocated. *out is set only on FDTD_OK.
 * Environment overrides read here (tuning and test aids; none changes the
 * bits): FDTD_ZCHUNKS and FDTD_SLAB_VARIANT (fused / slab z-split and tile
 * shape), FDTD_TZCHUNKS and FDTD_TEMPORAL_VARIANT (temporal sweep),
 * FDTD_NT_STORES = 0 / 1 (store policy; default: non-temporal when one sweep
 * streams more than 256 MB), FDTD_XCD_REMAP = 0 / 1 / 2 (workgroup-to-tile
 * order, read once per process: launch order; one contiguous block of tiles
 * per XCD; default 2, the temporal sweeps' resident workgroups covering one
 * contiguous tile range, which the slab sweeps treat as 1),
 * FDTD_TEMPORAL_SCHED = 0 / 1 (temporal sweeps, read once per process: one
 * workgroup per tile in the FDTD_XCD_REMAP order; default 1, one workgroup per
 * CU taking tiles from a queue).
 */
int fdtd_create(int nx, int ny, int nz, double dx, double dt, const fdtd_coef *coef,
                const fdtd_opts *opts, fdtd_t *out);

/*
 * Set the state to (E^0, H^{-1/2}) from six host arrays of type host_dtype
 * (FDTD_F64 or FDTD_F32) in the host layout above. Values are rounded to the
 * storage type (nearest even). Tangential E on the six walls is set to 0 (PEC)
 * whatever the input holds. Resets the step counter to 0. Host pointers are
 * read during the call only. Synchronous with respect to the host buffers.
 */
int fdtd_set_fields(fdtd_t h, const void *const host[6], int host_dtype);

/* As fdtd_set_fields, from six device buffers (same layout); enqueued on the solver's stream. */
int fdtd_set_fields_device(fdtd_t h, const void *const dev[6], int dev_dtype);

/*
 * Set the state to a seeded random (E^0, H^{-1/2}) on the device, the random
 * initial state of the cavity workloads (Fig. 1b, Sec. 4): every E node not
 * tangential to a wall takes 2u - 1 with u = (SplitMix64 output >> 11) 2^-53,
 * computed in FP64 and rounded once to the storage type (16-bit storage:
 * FP64 -> FP32 -> 16-bit). SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) is
 * used counter-style: output c of seed s is mix64(s + (c+1)*0x9E3779B97F4A7C15
 * mod 2^64), and component f (0 Ex, 1 Ey, 2 Ez) at linear index l of the host
 * layout uses counter (f << 40) + l. Tangential E on the walls and all H are
 * 0. Resets the step counter. Enqueued on the solver's stream (no wait).
 */
int fdtd_init_random(fdtd_t h, unsigned long long seed);

/*
 * Enqueue n >= 0 leapfrog steps (Sec. 2.1 algorithm listing: H update, H
 * boundary, E update, E boundary). Asynchronous: returns after launching.
 * The temporal schedule runs floor(n / tb) sweeps of tb steps and then one
 * sweep of n mod tb steps (16-bit storage rounds the state once per sweep).
 * Launch failures return FDTD_E_DEVICE at once; faults during execution
 * surface at the next fdtd_sync / fdtd_get_fields. The temporal sweeps hand
 * out tiles from counters in the solver's arena, which every launch leaves at
 * zero: launches on one solver must stay ordered on its stream (as they are
 * when issued through this call, also inside a captured graph that is
 * replayed on one stream); different solvers share nothing.
 */
int fdtd_step(fdtd_t h, long long n);

/*
 * fdtd_step for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops and harnesses that forbid allocation): the same
 * steps with the same bits, but the temporal sweeps take their scheduling
 * counters from a 256-byte array in the library's own device memory (one per
 * GPU, set up on the first call on that GPU) instead of the solver's arena,
 * which this call never touches beyond the field and coefficient boxes. It
 * calls no allocating routine. The counters are cleared by a small kernel on
 * the solver's stream at the start of every call (no hipMemsetAsync, so the
 * call can be captured). Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, other solvers) race and must be
 * ordered by the caller. Errors as fdtd_step (FDTD_E_DEVICE if the array's
 * address cannot be looked up).
 */
int fdtd_step_noalloc(fdtd_t h, long long n);

/*
 * Copy the current state (E^n, H^{n-1/2}) into six host arrays of type
 * host_dtype in the host layout above; waits for all enqueued work.
 */
int fdtd_get_fields(fdtd_t h, void *const host[6], int host_dtype);

/* As fdtd_get_fields, into six device buffers; enqueued on the solver's stream (no wait). */
int fdtd_get_fields_device(fdtd_t h, void *const dev[6], int dev_dtype);

/*
 * Copy the per-node coefficients into six host arrays of type host_dtype,
 * laid out like the fields: Ce for Ex, Ey, Ez and Ch for Hx, Hy, Hz (0 on
 * wall-tangential E and wall-normal H nodes, which never change). Values are
 * the storage-type numbers the kernels use.
 */
int fdtd_get_coefs(fdtd_t h, void *const host[6], int host_dtype);

/* Wait for all work enqueued on the solver's stream; reports deferred device faults. */
int fdtd_sync(fdtd_t h);

/* Number of leapfrog steps applied since the last set_fields (-1 for an invalid handle). */
long long fdtd_steps_done(fdtd_t h);

/* Diagnostics computed in FP64 on the device from the stored fields; waits. */
enum {
    FDTD_DIAG_ENERGY = 0,   /* W = sum E^2/Ce + sum H^{n-1/2} H^{n+1/2}/Ch (conserved exactly in exact arithmetic) */
    FDTD_DIAG_SUM_E2 = 1,   /* sum of E^2 over all E nodes */
    FDTD_DIAG_SUM_H2 = 2,   /* sum of H^2 over all H nodes */
    FDTD_DIAG_MAX_DIVB = 3, /* max over cells of |div (H/Ch)| (wall-normal H counted as 0) */
    FDTD_DIAG_MAX_ETAN = 4, /* max |tangential E| on the six walls (0 under PEC) */
    FDTD_DIAG_NONFINITE = 5,/* number of non-finite field values */
    FDTD_DIAG_N = 6
};
int fdtd_diag(fdtd_t h, double out[FDTD_DIAG_N]);

/*
 * Resolved configuration: out[0] kernel, out[1] steps per sweep, out[2]
 * storage dtype, out[3] sweeps launched since create, out[4] per-node Ce (1/0),
 * out[5] per-node Ch (1/0), out[6] padded x pitch, out[7] device bytes used.
 */
int fdtd_query(fdtd_t h, long long out[8]);

/*
 * Schedule of fdtd_step: which kernel, its steps per sweep, tile shape and
 * z-split. For FP32 and FP64 storage every schedule gives the same bits, so
 * choosing one changes only speed. 16-bit storage rounds the state at the end
 * of every sweep: there the steps per sweep are part of the numerics (the
 * same tb_steps gives the same bits whatever the kernel's tiling).
 */
typedef struct {
    int kernel;         /* FDTD_KERNEL_PLAIN .. FDTD_KERNEL_TEMPORAL */
    int tb_steps;       /* steps per sweep (temporal: 1..4, 1..3 for variant 1; others 1) */
    int variant;        /* tile shape: slab 0..3 = (cells per lane, waves) (2,16) (2,8) (1,16) (1,8);
                           temporal 0..1 = 64 columns x 2 rows per wave, 128 columns x 1 row per wave */
    int zchunks;        /* z-ranges per launch (fused, slab, temporal), 1..nz */
    double ms_per_step; /* fdtd_autotune results: measured milliseconds per leapfrog step */
} fdtd_schedule;

/* The schedule fdtd_step uses now. */
int fdtd_get_schedule(fdtd_t h, fdtd_schedule *out);

/* Use this schedule from now on (FDTD_E_ARG / FDTD_E_UNSUPPORTED for a combination not built). */
int fdtd_set_schedule(fdtd_t h, const fdtd_schedule *sched);

/*
 * Time every built schedule on this solver (its grid, storage and
 * coefficients: tile sizes, steps per sweep and z-split; the search the
 * paper leaves as future work, Sec. 7; 16-bit storage keeps its steps per
 * sweep and searches the tiling only) for trial_steps steps each (0: 6;
 * rounded up to whole sweeps) after one warm-up sweep, and keep the fastest.
 * The state and the step count are restored afterwards (a copy of the six
 * field boxes is held in a temporary device allocation during the call).
 * results (may be NULL) receives up to max_results schedules in the order
 * tried, each with ms_per_step; *n_results (may be NULL) the number tried.
 */
int fdtd_autotune(fdtd_t h, int trial_steps, fdtd_schedule *results, int max_results, int *n_results);

/* The hipStream_t the solver enqueues on. */
void *fdtd_stream(fdtd_t h);

/* Release device memory the library allocated (not a caller arena) and the handle. */
int fdtd_destroy(fdtd_t h);

/*
 * ---- Adjoint: gradient of a driven-cavity probe objective ----
 *
 * Ampere's law of Sec. 2 (Eq. 2) carries a current density that the
 * source-free cavity update drops; here it drives the cavity as a point
 * source. Starting from the solver's current state (E^0, H^{-1/2}), each of
 * the N steps is a leapfrog step (Sec. 2.1 algorithm listing), then w[n-1] is
 * added to the source node, then the probe nodes are read:
 *     J = sum_{n=1..N} sum_p (E^n at probe p)^2.
 * fdtd_adjoint_backward returns dJ/d eps_r per cell by the discrete adjoint:
 * the same curl stencils run in reverse time with the coefficient inside the
 * curl (the E curl is minus the transpose of the H curl), accumulating
 * dJ/dCe = sum_n lam^{n+1} (L H^{n+1/2}) per edge in FP64 (with FP32
 * storage the terms are first summed in FP32 over fixed groups of 16 steps,
 * n = 16m .. 16m+15, independent of the checkpoint interval), then
 * dJ/d eps_cell = sum over the cell's 12 edges of dJ/dCe * (-Ce^2 dx/dt / 4)
 * (Ce = dt/(dx * mean eps of the edge's four cells)). The forward pass stores
 * (E^n, H^{n-1/2}) every K = checkpoint_every steps and keeps H^{n+1/2} of
 * every step of the last segment; the backward pass recomputes each other
 * segment from its checkpoint (checkpoint-and-recompute), so device memory is
 * ceil(N/K) states + min(K, N) H-fields (+ two adjoint states, the FP64
 * gradient boxes and, with FP32 storage, their FP32 group sums). With K >= N
 * nothing is recomputed: the backward costs one reverse sweep per step.
 * checkpoint_every = 0 picks K = N when that memory is at most half of the
 * device's free memory (and within FDTD_HBM_BUDGET bytes when that is set),
 * else K = ceil(sqrt(2N)), the interval of least memory. Every K gives the
 * same bits.
 * Each forward and recompute step is one slab sweep that also adds the source
 * and (up to 16 probes) records the probes; each reverse step is one fused
 * sweep (mu' = mu - K(Ce lam), the gradient terms, lam' = lam - L(Ch mu'),
 * the probe terms) from one adjoint buffer to the other. Environment aids
 * (none changes the bits): FDTD_ADJ_FUSED = 0 (the one-cell-per-thread
 * reverse kernels, in place), FDTD_ADJ_VARIANT = 0..3 (tile shape of the
 * fused sweep; default 1), FDTD_ADJ_ZCHUNKS (its z-split).
 */
typedef struct fdtd_adjoint *fdtd_adjoint_t;

typedef struct {
    int src_field;            /* E component of the source node (FDTD_EX..FDTD_EZ), or -1 for none */
    int src_i, src_j, src_k;  /* source node, interior (not tangential to a wall) */
    const double *waveform;   /* nsteps values; waveform[n-1] is added after the E update of step n */
    int nprobes;              /* 0 .. 4096 */
    const int *probes;        /* 4 ints per probe: E component, i, j, k (interior E nodes) */
    long long nsteps;         /* N >= 1 */
    int checkpoint_every;     /* K >= 1, or 0: automatic (K = N when it fits, see above) */
} fdtd_adjoint_problem;

/*
 * Bind an adjoint problem to a solver created with per-cell eps_r (FP32 or
 * FP64 storage; FDTD_E_UNSUPPORTED otherwise). Host arrays are copied.
 * Allocates the checkpoint, history and adjoint buffers (FDTD_E_NOMEM). The
 * solver must outlive the handle; it is not thread-safe with it.
 */
int fdtd_adjoint_create(fdtd_t solver, const fdtd_adjoint_problem *problem, fdtd_adjoint_t *out);

/* Run the N driven steps from the solver's current state, storing checkpoints; *J receives J. Waits. */
int fdtd_adjoint_forward(fdtd_adjoint_t adj, double *J);

/*
 * Reverse pass of the last forward: grad_eps receives dJ/d eps_r per cell
 * (host, nx*ny*nz doubles, x-fastest). lam0, if not NULL, receives dJ/dE^0
 * (three host arrays in the Ex, Ey, Ez host layout, lam0_dtype FDTD_F32 or
 * FDTD_F64). The solver's state afterwards is the forward's starting state
 * (E^0, H^{-1/2}; the recompute borrows its buffers); its step count is left
 * as the forward left it. Waits.
 */
int fdtd_adjoint_backward(fdtd_adjoint_t adj, double *grad_eps, void *const lam0[3], int lam0_dtype);

/* Free the adjoint buffers (waits for the solver's stream). */
int fdtd_adjoint_destroy(fdtd_adjoint_t adj);

/*
 * ---- Serving pool: continuous batching of many cavity solves ----
 *
 * A pool owns one block of device memory (hbm_budget bytes) and a host thread
 * that runs the request loop. Submitted requests wait in a queue until their
 * state fits the free memory (first fit; FIFO unless backfill is set, which
 * lets a later request that fits pass one that does not). Admitted requests
 * keep their fields resident; each loop round advances every admitted request
 * by min(tb_steps, steps left) leapfrog steps (the Sec. 2.1 algorithm
 * listing) in ONE temporal-sweep launch over the tiles of all of them (one
 * launch per distinct (steps, per-node Ce, per-node Ch) group). A request
 * leaves the batch after its last step; new requests join at the next round.
 * Per-request arithmetic is the single-solve tile code on its own buffers, so
 * a request gives the same bits alone and in any mix, and the same bits as an
 * FP32 fdtd_t solver with the same dims, coefficients, initial state and
 * steps. Storage is FP32.
 *
 * Timing: t_submit, t_admit, t_done are host steady-clock seconds since pool
 * creation; t_done is when the loop thread observed the completion event
 * recorded after the request's last sweep (it waits on launches in order, so
 * the observation trails the device by at most one batched launch).
 */
typedef struct fdtd_pool *fdtd_pool_t;

typedef struct {
    size_t hbm_budget; /* device bytes for request state (>= 1 MiB); with arena: its size */
    int device;        /* HIP device ordinal */
    int tb_steps;      /* steps per batched sweep, 1..4 (0: 4; requests with per-node Ch take at most 3) */
    int max_active;    /* most admitted requests at once, 1..65536 (0: 256) */
    int backfill;      /* 0: strict FIFO admission; 1: requests that fit may pass the queue head */
    void *stream;      /* hipStream_t for all request work; NULL: the pool creates one */
    void *arena;       /* caller-owned device memory of hbm_budget bytes; NULL: hipMalloc */
} fdtd_pool_opts;

typedef struct {
    int nx, ny, nz;              /* cells, each >= 2 */
    double dx, dt;               /* as fdtd_create (Courant limit checked) */
    long long steps;             /* leapfrog steps, >= 0 */
    const double *eps_r, *mu_r;  /* per-cell materials as fdtd_coef (NULL: 1); copied at submit */
    const void *const *fields;   /* NULL: seeded state as fdtd_init_random(seed); else six host
                                    arrays (host layout, fields_dtype) copied at submit */
    int fields_dtype;            /* FDTD_F32 or FDTD_F64 when fields != NULL */
    unsigned long long seed;
    int keep;                    /* 1: the final state stays resident until fdtd_pool_fetch /
                                    fdtd_pool_release; 0: its memory is reused at completion */
} fdtd_request;

typedef enum {
    FDTD_REQ_QUEUED = 0,   /* waiting for memory */
    FDTD_REQ_ACTIVE = 1,   /* admitted; sweeps enqueued or pending */
    FDTD_REQ_DONE = 2,     /* all steps finished on the device */
    FDTD_REQ_RELEASED = 3, /* released (or cancelled while queued) */
    FDTD_REQ_FAILED = 4    /* the pool hit a device error */
} fdtd_request_state;

typedef struct {
    int state;                        /* fdtd_request_state */
    double t_submit, t_admit, t_done; /* seconds since pool creation; -1 if not reached */
    long long steps;
    size_t bytes;                     /* device bytes held while admitted */
} fdtd_request_info;

typedef struct {
    long long submitted, completed, queued, active;
    long long launches;        /* batched launches enqueued */
    long long request_sweeps;  /* (request, sweep) pairs enqueued */
    double cell_updates;       /* cell-steps enqueued */
    size_t bytes_used, bytes_peak, budget;
    int peak_active;           /* most requests admitted with sweeps left at once */
    int failed;
} fdtd_pool_counters;

/* Defaults: tb_steps 4, max_active 256, backfill 0, device 0; hbm_budget must be set. */
int fdtd_pool_opts_default(fdtd_pool_opts *opts);

/* Device bytes a request holds while admitted (fields double-buffered, per-node
   coefficients, and an FP64 staging array when it has host inputs or keep = 1). */
int fdtd_pool_request_bytes(const fdtd_request *req, size_t *out);

/* Create a pool and start its loop thread. FDTD_E_NOMEM if the budget cannot be allocated.
   Each batched launch cuts every request into z-chunks of about 64 planes (32 when the
   launch would have fewer than 512 tiles); FDTD_POOL_CHUNK (8..4096, read once per
   process) sets the length. The pool also allocates its tile-queue counters (256 bytes)
   outside the budget. */
int fdtd_pool_create(const fdtd_pool_opts *opts, fdtd_pool_t *out);

/*
 * Queue a request; *id is its number (0, 1, 2, ... in submit order). Checks
 * as fdtd_create (FDTD_E_ARG, FDTD_E_CFL) and FDTD_E_NOMEM if the request can
 * never fit the budget. Host arrays are copied during the call. Thread-safe.
 */
int fdtd_pool_submit(fdtd_pool_t pool, const fdtd_request *req, long long *id);

/*
 * Block until request id is done (id >= 0) or until every submitted request
 * has left the queue and the device (id = -1). timeout_s < 0 waits without
 * limit; otherwise FDTD_E_TIMEOUT when it runs out. FDTD_E_DEVICE if the pool
 * failed. A queued request behind kept results that are never released waits
 * for ever. Thread-safe.
 */
int fdtd_pool_wait(fdtd_pool_t pool, long long id, double timeout_s);

/* State and timestamps of request id. Thread-safe. */
int fdtd_pool_info(fdtd_pool_t pool, long long id, fdtd_request_info *out);

/*
 * Copy the final state (E^n, H^{n-1/2}) of a done keep = 1 request into six
 * host arrays (host layout, FDTD_F32 or FDTD_F64); waits for the copy. The
 * request stays resident until fdtd_pool_release. Thread-safe: while a fetch
 * of a request runs, fdtd_pool_release of the same id returns FDTD_E_STATE.
 */
int fdtd_pool_fetch(fdtd_pool_t pool, long long id, void *const host[6], int host_dtype);

/* Free a request's memory (done requests) or cancel it (queued). FDTD_E_STATE while admitted and
 * running, or while a fetch of it is in progress. Thread-safe. */
int fdtd_pool_release(fdtd_pool_t pool, long long id);

/* Counters of the pool. Thread-safe. */
int fdtd_pool_stats(fdtd_pool_t pool, fdtd_pool_counters *out);

/* Stop the loop, wait for enqueued device work, free everything. Queued requests are dropped. */
int fdtd_pool_destroy(fdtd_pool_t pool);

/*
 * Measurement helper (not part of the method): enqueue a plain 16-byte-wide
 * streaming copy of `bytes` bytes from src to dst (device pointers, 16-byte
 * aligned, bytes a multiple of 16) on `stream` (hipStream_t or NULL). It
 * reads and writes a known number of bytes, which gives the achievable HBM
 * bandwidth and calibrates hardware memory counters. FDTD_E_ARG on a bad
 * pointer or size, FDTD_E_DEVICE if the launch fails.
 */
int fdtd_probe_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Static text for a status code. */
const char *fdtd_strerror(int status);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *fdtd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_H */
