/*
 * holb.h -- C ABI of the high-order lattice Boltzmann library for AMD
 * Instinct MI355X (gfx950).
 *
 * The library advances the shifted BGK lattice Boltzmann equation with
 * Hermite-polynomial source terms of Li et al., "Constructing the body
 * source for high-order lattice Boltzmann method" (arXiv:2411.10751):
 *
 *   f^_i(x + c_i, t + 1) - f^_i(x, t) = -(f^_i - f^eq_i) / tau_hat
 *                                      + (1 - 1 / (2 tau_hat)) S_i     (Eq. 4.4)
 *
 * on the D2Q37 or D3Q39 multispeed lattice (Section 4.1), with the
 * fourth-order Hermite equilibrium f^eq (Eq. 2.2) and the source
 * S_i = F_i + H_i + P_i made of the body force (Eq. 3.3), the thermal-
 * dissipation correction that sets the Prandtl number (Eq. 3.7) and the
 * pressure-tensor source of the pseudopotential multiphase model (Eqs. 3.8,
 * 3.12).  Macroscopic fields follow the shifted moments of Eq. (4.5).
 *
 * Conventions
 *  - Lattice units: dt = dx = 1.  Velocities u are lattice velocities
 *    (Table 2 form); temperature theta is 1 at the lattice reference
 *    temperature, so the isothermal sound speed squared is c0^2 theta.
 *  - Fields are structure-of-arrays in device memory, float32:
 *    rho[N], u[D][N], theta[N], with cell = x + nx * (y + ny * z),
 *    N = nx * ny * nz (nz = 1 for D2Q37).
 *  - Every call returns a holb_status; no exception crosses the ABI.  On
 *    failure holb_last_error() returns a thread-local message.
 *  - Ownership: the caller allocates all device memory (the workspace and
 *    every field buffer) and keeps it alive until *_destroy; the library
 *    allocates none.  Handles are host objects freed by *_destroy.
 *  - Streams: all GPU work of a handle is ordered on the HIP stream given at
 *    creation (NULL = the default stream).  One handle must not be used from
 *    two threads at once.
 */
#ifndef HOLB_H
#define HOLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HOLB_ABI_VERSION 4

typedef int32_t holb_status;
#define HOLB_OK 0
#define HOLB_EINVAL (-1)       /* bad argument or configuration value */
#define HOLB_ESIZE (-2)        /* buffer or workspace too small / misaligned */
#define HOLB_EHIP (-3)         /* a HIP runtime call failed */
#define HOLB_ENUMERIC (-4)     /* the device raised a numeric error (see holb_error_flags) */
#define HOLB_EUNSUPPORTED (-5) /* valid values, combination not supported */
#define HOLB_ESTATE (-6)       /* call out of order (e.g. step before init) */

/* Lattices (Section 4.1). */
#define HOLB_D2Q37 0
#define HOLB_D3Q39 1

/* Source-term mask. */
#define HOLB_SRC_BODY 1u    /* body force F = rho g, Eq. (3.3) */
#define HOLB_SRC_THERMAL 2u /* thermal-dissipation source H_i, Eq. (3.7) */
#define HOLB_SRC_PTENSOR 4u /* pseudopotential force (Eq. 3.8) + P_i (Eq. 3.12) */

/* Population storage in device memory.  Arithmetic is always FP32.
 * Populations are stored as deviations, divided by w_i, from the rest
 * equilibrium of a frame (a density and temperature): the frame of their cell
 * or of their plane, per the frame mode below.  The 16-bit forms also
 * subtract the bracket of the uniform background velocity u0 and round to
 * nearest-even (see holb_get_state for the exact format). */
/* Frames (the reference the stored populations are deviations from, see
 * holb_get_state).  CELL keeps each cell's density and temperature of the
 * last step beside its populations (4 bytes per cell, read with every pull).
 * PLANE keeps one fixed frame per plane along the last axis (the plane means
 * of the initial fields): nothing per cell, and suited to states whose
 * density and temperature vary mostly along that axis -- it keeps less of the
 * precision where the state drifts far from those means.  CELL_U (16-bit
 * storage only) adds the cell's momentum to its frame,
 * so that the stored deviations lose their first-order velocity part as well:
 * about 3x smaller BF16 errors in flows with O(0.05) velocities, for a second
 * round of Q - 1 loads per pull (at 256^3 about 1.5x the step time of CELL).
 * AUTO picks PLANE for FP32 and FP16 storage with walls (which impose the
 * mean profile along the wall-normal axis) and for FP32 and FP16 in a
 * periodic domain without the pressure-tensor source (without frame words the
 * pull is 8-10% faster in FP32 and 20% faster in FP16 on the body-force
 * workload, whose FP16 errors are those of CELL), except CELL_U for FP16 with
 * the thermal source in a periodic domain; CELL with the pressure-tensor
 * source in a periodic domain (liquid and vapour in one plane: about 20x the
 * error with PLANE in FP32), for BF16 with walls and for BF16 in a periodic
 * domain.  A state with a jump along the last axis across a periodic boundary
 * (a ramp wrapped around), or with density or temperature varying strongly
 * within the planes, keeps more precision with CELL.
 * Accuracy of the 16-bit forms against the FP64 oracle (relative L-infinity,
 * bound 2e-3): FP16 meets it on every workload tested at its horizon with
 * these frames, except a flat liquid slab over 1000 steps (u 2.5e-3 against
 * the 0.01 c0 velocity floor); BF16 meets it on the walled Rayleigh-Benard
 * boxes (u 1.75e-3 on 64^3 over 2000 steps) but not on the droplet workload
 * (u 6e-3 to 1e-2) or the thermal workload at 20,000 steps (u 4.6e-2), with
 * any frames: use FP16 or FP32 storage there. */
#define HOLB_FRAMES_AUTO 0
#define HOLB_FRAMES_CELL 1
#define HOLB_FRAMES_PLANE 2
#define HOLB_FRAMES_CELL_U 3

/* Equation of state of the pseudopotential (HOLB_SRC_PTENSOR), parameters
 * eos_a, eos_b, eos_T: van der Waals p = rho T / (1 - b rho) - a rho^2, or
 * Carnahan-Starling (Section 5.4, Eq. 5.9, R_g = 1)
 * p = rho T (1 + e + e^2 - e^3) / (1 - e)^3 - a rho^2 with e = b rho / 4. */
#define HOLB_EOS_VDW 0
#define HOLB_EOS_CS 1

#define HOLB_STORE_F32 0
#define HOLB_STORE_F16DEV 1
#define HOLB_STORE_BF16DEV 2

/* Device error flags (holb_error_flags). */
#define HOLB_ERR_DENSITY 1u  /* rho <= 0 or not finite */
#define HOLB_ERR_THETA 2u    /* theta <= 0 or not finite */
#define HOLB_ERR_EOS 4u      /* psi^2 < 0 or b rho >= 1 in the equation of state */
#define HOLB_ERR_WALL 8u     /* the wall-node target of the TMS closure did not converge */

typedef struct {
    int32_t abi_version;  /* must equal HOLB_ABI_VERSION */
    int32_t lattice;      /* HOLB_D2Q37 or HOLB_D3Q39 */
    int32_t nx, ny, nz;   /* grid; nz = 1 for D2Q37 */
    double tau_hat;       /* shifted relaxation time, > 0.5 (Eq. 4.3); nu = c0^2 theta (tau_hat - 1/2) */
    uint32_t sources;     /* HOLB_SRC_* mask */
    int32_t isothermal;   /* 1: theta held at 1 (multiphase mode of Section 5.4) */
    double g[3];          /* body-force acceleration, F = rho g (HOLB_SRC_BODY) */
    double prandtl;       /* Prandtl number of H_i (HOLB_SRC_THERMAL), > 0 */
    double eos_a, eos_b, eos_T; /* parameters a, b, T of the equation of state (eos) */
    double sc_G;          /* pseudopotential coupling G (the paper uses -1) */
    double ptensor_k;     /* free parameter k of P_i, Eq. (3.12), evaluated in Hermite units: the
                           * paper's Carnahan-Starling optimum 3.02 is 3.02 c0^4 here */
    int32_t storage;      /* HOLB_STORE_* */
    double rho0, theta0, u0[3]; /* background state: u0 (with rho0, theta0) centres the 16-bit
                                 * storage; theta0 is the offset of the temperature field of
                                 * the gradient stencil */
    int32_t walls;        /* 0: periodic; 1: TMS walls (Section 4.3, Eqs. 4.7-4.8) normal to the
                           * last axis.  The first and last layers hold the wall nodes, outside the
                           * fluid; each wall lies half-way between them and the next layer, so the
                           * fluid is n - 2 nodes high.  A wall node's target is solved from the
                           * wall's boundary conditions: no net mass through the wall, and after the
                           * closure the node holds the reflection of the first fluid node's
                           * tangential velocity and temperature about the wall values. */
    double theta_wall[2]; /* wall temperatures: [0] at index 0, [1] at index n-1 */
    double u_wall[2][3];  /* wall velocities, same order */
    int32_t frames;       /* HOLB_FRAMES_*: reference of the stored populations */
    int32_t eos;          /* HOLB_EOS_*: equation of state of the pseudopotential */
    int32_t grad_lag;     /* thermal source: time level of theta in the gradient of H_i (Eq. 3.7;
                           * Section 3.2 does not fix it): 0 = the same step's theta (a second
                           * pass over the populations per step), 1 = the previous step's theta,
                           * which the collision writes out as it goes (one pass per step; before
                           * the first step, the initial state's theta).  Single runs only. */
} holb_config;

typedef struct holb_sim holb_sim;
typedef struct holb_batch holb_batch;

/* Thread-local description of the last failure in this thread. */
const char* holb_last_error(void);

/* Velocity set used by the library (Section 4.1): Q, D, c[Q][3] (int),
 * w[Q], c0^2.  Any output pointer may be NULL.  c/w need room for 39. */
holb_status holb_lattice_info(int32_t lattice, int32_t* Q, int32_t* D, int32_t* c, double* w,
                              double* c0sq);

/* Bytes of device workspace a configuration needs (two population buffers,
 * stencil fields, wall targets, reduction partials).  Pure host call. */
holb_status holb_workspace_size(const holb_config* cfg, size_t* bytes);

/* Validate cfg and bind a caller-owned device workspace (256-byte aligned,
 * at least holb_workspace_size bytes) and stream.  Pure host call: launches
 * nothing.  Errors: HOLB_EINVAL (values, tau_hat <= 0.5, dims), HOLB_ESIZE
 * (workspace, or more than 2^29 cells), HOLB_EUNSUPPORTED (e.g. thermal source with isothermal=1,
 * pressure tensor without isothermal=1 or with walls). */
holb_status holb_create(const holb_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream,
                        holb_sim** out);

/* Set the initial state f^0 = f^eq(rho, u, theta) from device fields
 * (rho[N], u[D][N], theta[N]; theta ignored when isothermal).  The first
 * holb_step then performs the t = 0 collision with the source terms.
 * Asynchronous. */
holb_status holb_init(holb_sim* s, const float* rho, const float* u, const float* theta);

/* Advance n >= 0 time steps of Eq. (4.4) (wall closure, shifted moments,
 * sources, BGK collision, streaming).  Asynchronous on the stream.  Runs of
 * 16 steps go as one replay of a HIP graph (captured on a library-owned
 * stream at the first such call, again after the kernel variant changes);
 * the rest, and every step while holb_timing_start is active, are launched
 * one by one.  Both give the same bits.  With walls a step forks its wall
 * work (the closure solve) onto a second, library-owned stream of default
 * priority (created at the first call) and makes the caller's stream wait
 * for it within the same step: work queued on the caller's stream afterwards
 * sees the whole step.  The library-owned streams are created on the device
 * that is current at that first call, which must be the simulation's. */
holb_status holb_step(holb_sim* s, int64_t n);

/* Macroscopic fields of the current state (Eq. 4.5) into device buffers
 * rho[N], u[D][N], theta[N] (any may be NULL).  Synchronises the stream and
 * returns HOLB_ENUMERIC if the device error flags are set. */
holb_status holb_fields(holb_sim* s, float* rho, float* u, float* theta);

/* Global FP64 totals of the current state (the conserved moments of Eq. 2.3,
 * with the macroscopic fields of Eq. 4.5) into host out[5]: mass sum rho,
 * momentum sum rho u (x, y, z; z = 0 in 2D), energy
 * sum (rho |u|^2 + rho D c0^2 theta) / 2.  Deterministic order.  Synchronises;
 * returns HOLB_ENUMERIC if the device error flags are set. */
holb_status holb_reduce(holb_sim* s, double out[5]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): holb_reduce
 * with its FP64 block partials and totals kept in a library-owned static
 * device array (about 5 MB per GPU, held until the process ends) instead of
 * the workspace.  Same kernels and partition, so the totals are bitwise those
 * of holb_reduce.  Grids of more than HOLB_NOALLOC_MAX_CELLS cells are
 * rejected with HOLB_ESIZE.  All calls on one GPU share the array: calls that
 * overlap on one GPU (other threads, other streams) race.  Allocates nothing;
 * synchronises; HOLB_ENUMERIC if the device error flags are set. */
#define HOLB_NOALLOC_MAX_CELLS 33554432
holb_status holb_reduce_noalloc(holb_sim* s, double out[5]);

/* Device error flags (HOLB_ERR_*) raised since creation; synchronises. */
holb_status holb_error_flags(holb_sim* s, uint32_t* flags);

/* Raw population state: size in bytes, and device-to-device copies out of /
 * into the library's current buffer.  Layout: Q planes of 256-byte aligned
 * pitch (element type per storage, velocity order of holb_lattice_info),
 * then the frames:
 *   CELL:   one 32-bit word per cell, binary16 rho_F in the low half and
 *           binary16 theta_F - 1 in the high half (padded to 256 bytes);
 *   CELL_U: that plane, then a second plane (also padded to 256 bytes)
 *           of one momentum word per cell, P = rho_F (u_F - u0) / c0^2 as
 *           three 10-bit two's-complement multiples of 2^-10 (bits 0-9 x,
 *           10-19 y, 20-29 z);
 *   PLANE:  no per-cell words; after the planes (256-byte aligned) a float
 *           table of (rho_F, theta_F - 1) per plane along the last axis,
 *           then R_s(plane m - c_m) - R_s(plane m) at [(m 7 + c_m + 3) NS + s].
 * With walls, the wall targets follow (again 256-byte aligned): for the
 * three layers next to each wall (layer k = 0, 1, 2 from the low wall, then
 * n-3, n-2, n-1), the last step's rho, u[D] and theta, each a plane of the
 * layer's cells (double); then, for the low and the high wall, the wall-node
 * target the last step solved (rho, u[D], theta, planes of the layer's cells:
 * the starting point of the next solve); then, per wall, the 16 LU factors of
 * the Jacobian that solve used (4 x 4 row-major, each a plane of the layer's
 * cells; all zero before the first step).  Restoring them makes a resumed
 * walled run continue bitwise as the uninterrupted one.  Slots of the first
 * three layers whose population would leave through a wall are pulled by no
 * node: they hold the outflow whose mass the next closure gives back.  holb_set_state needs no
 * holb_init before it and clears the device error flags.
 * Slot i of cell y holds the post-collision population f*_i(y) of the last
 * step in the frame F of y: h = f*_i / w_i - rho_F (1 + t_i(u = 0, theta_F))
 * of Eq. (2.2) (CELL_U: minus c_i . P as well) in FP32 storage, h - d_i
 * rounded to nearest-even in the 16-bit format otherwise, with
 * d_i = (f^eq_i(rho0, u0, theta0) - f^eq_i(rho0, 0, theta0)) / w_i; pulling
 * slot i of y = x - c_i gives the pre-collision population of x.  The format
 * is the library's own: copy it back only into a simulation of the same
 * configuration. */
holb_status holb_state_bytes(holb_sim* s, size_t* bytes);
holb_status holb_get_state(holb_sim* s, void* dev_dst, size_t bytes);
holb_status holb_set_state(holb_sim* s, const void* dev_src, size_t bytes);

/* Pick the fastest kernel variant for this configuration by timing each
 * candidate on trial steps that leave the state untouched (the fastest of
 * three timings of 4 steps, taken in round-robin passes); results are
 * bitwise identical across variants.  Synchronises.  variant_out may be NULL. */
holb_status holb_tune(holb_sim* s, int32_t* variant_out);
/* Force a kernel variant (0 = the default); HOLB_EUNSUPPORTED if it does not
 * apply to this configuration.  holb_num_variants reports how many exist.
 * Variants are orders in which blocks take cells (the eight XCDs receive
 * blocks round-robin, each with its own L2): 0 cell order, 1 a contiguous
 * eighth of the cells per XCD, 2 the chip sweeping plane by plane with each
 * XCD taking a band of an eighth of the plane, 3, 4, 5 the same with bands of
 * 4, 8, 16 blocks of 256 cells.  An order that does not divide the grid
 * evenly falls back to cell order. */
holb_status holb_set_variant(holb_sim* s, int32_t variant);
holb_status holb_num_variants(holb_sim* s, int32_t* n);

/* Instrumentation.  holb_timing_start makes each of the next max_steps
 * (1..100000) steps record a pair of HIP events on the library's stream
 * around the step's dominant kernel (the collision of the cells away from the
 * wall layers; in a periodic domain, of every cell).  holb_timing_stop
 * synchronises on the last event and returns the summed kernel time in ms,
 * the number of timed launches, the cells one launch updates and the kernel's
 * name as a profiler lists it, without namespace and spaces (written to
 * kernel, at most kernel_len bytes with the terminator; any output may be
 * NULL).  Steps beyond max_steps run untimed; holb_timing_start again
 * discards the events of an unfinished timing. */
holb_status holb_timing_start(holb_sim* s, int32_t max_steps);
holb_status holb_timing_stop(holb_sim* s, double* kernel_ms, int64_t* launches, int64_t* cells_per_launch,
                             char* kernel, size_t kernel_len);

holb_status holb_destroy(holb_sim* s);

/* ---- Batched form: many independent periodic D2Q37 runs in one launch ---- */

/* Every run uses its own grid (nx, ny), tau_hat, sources, g and Pr; all runs
 * share lattice (D2Q37), storage (HOLB_STORE_F32), isothermal = 0, walls = 0,
 * per-plane frames, the thermal source on or off, and grad_lag.  A step is
 * the temperature pass and the collision pass over all runs (two launches);
 * with grad_lag = 1 (thermal source: the previous step's temperature
 * gradient) it is the collision pass alone, which also writes the
 * temperature field for the next step. */
holb_status holb_batch_workspace_size(const holb_config* cfgs, int32_t n_runs, size_t* bytes);
holb_status holb_batch_create(const holb_config* cfgs, int32_t n_runs, void* dev_workspace,
                              size_t bytes, void* hip_stream, holb_batch** out);
/* rho/u/theta: host arrays of n_runs device pointers, fields laid out per run. */
holb_status holb_batch_init(holb_batch* b, const float* const* rho, const float* const* u,
                            const float* const* theta);
/* n steps of every run; runs of 16 steps are replayed from a captured HIP
 * graph (one per starting buffer), the rest launched one by one. */
holb_status holb_batch_step(holb_batch* b, int64_t n);
holb_status holb_batch_fields(holb_batch* b, int32_t run, float* rho, float* u, float* theta);
holb_status holb_batch_reduce(holb_batch* b, int32_t run, double out[5]);
/* Launch shape of the batched kernels.  Variant v in [0, 12) splits every
 * run into work items of 256 << (v / 3) consecutive cells (256 to 2048; a
 * block takes an item 256 cells at a time) and runs a persistent grid of 4, 8
 * or 2 blocks per compute unit (v % 3) over the work list; 0 is the default.
 * Results are bitwise identical across variants.  holb_batch_set_variant
 * uploads the work list of the new item size on the handle's stream and
 * synchronises it (HOLB_EUNSUPPORTED outside [0, 12)).  holb_batch_tune times
 * every variant on trial steps (they write the idle buffer, so the state is
 * unchanged; the fastest of three timings of 4 steps, taken in round-robin
 * passes), keeps the fastest and returns it in variant_out (may be NULL); it
 * synchronises and needs holb_batch_init first (else HOLB_ESTATE). */
holb_status holb_batch_tune(holb_batch* b, int32_t* variant_out);
holb_status holb_batch_set_variant(holb_batch* b, int32_t variant);
/* Instrumentation, as holb_timing_start / holb_timing_stop: while a timing is
 * open, holb_batch_step runs its steps eagerly (no graph replay) and records
 * a pair of HIP events around each collision launch (k_batch_step, all runs;
 * cells_per_launch is the total cell count of the batch). */
holb_status holb_batch_timing_start(holb_batch* b, int32_t max_steps);
holb_status holb_batch_timing_stop(holb_batch* b, double* kernel_ms, int64_t* launches, int64_t* cells_per_launch,
                                   char* kernel, size_t kernel_len);
holb_status holb_batch_destroy(holb_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* HOLB_H */
