/*
 * vlbm.h - C ABI of the MI355X (gfx950) vectorial lattice Boltzmann library.
 *
 * Method: Hosseini & Karlin, "Vectorial lattice Boltzmann solver for
 * compressible inviscid flows with generic equation of state",
 * arXiv 2609.10639.  One time step of the library is the paper's fused lattice
 * update: moments W = sum_i f_i (Sec. III.A), EOS closure (Sec. II.C,
 * Eqs. 13, 15-17), CFL retargeting of the link speed with exact moment
 * reprojection (Sec. III.E, Eqs. 36-40), the Ducros-gated adaptive relaxation
 * coefficient beta(x,t) (Sec. III.D, Eqs. 28-35), over-relaxation towards the
 * flux-consistent vector equilibrium (Eqs. 20, 22), exact transport (Eq. 21)
 * and the global max(|u_alpha| + c_s) reduction that feeds the next step.
 *
 * Conventions
 *   - Lattices: D1Q2 (dim = 1) and D2Q4 (dim = 2).  Directions are ordered
 *     (+x, -x, +y, -y); components (rho, rho u, [rho v,] rho E).
 *   - Macroscopic arrays W are FP64, structure-of-arrays, shape
 *     (dim+2, ny, nx), x fastest; ny == 1 in 1-D.  Cell centres at (j+1/2) dx.
 *   - Populations live on the device in the precision chosen at creation
 *     (FP64 or FP32): dim+2 component planes for each of the 2*dim directions,
 *     plane index i*(dim+2)+k, each plane padded to `vlbm_plane_elems`.
 *   - Every call is ordered on the HIP stream given in the config (NULL = the
 *     default stream).  Calls that return host data synchronise that stream.
 *   - Pointers flagged *_on_device are device pointers the caller owns; they
 *     are only borrowed for the duration of the call (stream-ordered).
 *   - Errors are returned as vlbm_status; no call aborts the process.  A
 *     failing call leaves a message readable with vlbm_last_error().
 *
 * Readings of points the paper leaves open (identical in the CPU oracle):
 *   - initial populations are the equilibrium at c0 = s_max(W0)/CFL;
 *   - the final step of vlbm_run_to_time shortens dt to t_end - t, which is a
 *     retarget to c = dx/(t_end - t) with reprojection; it triggers when
 *     t + dt >= t_end (1 - 1e-14) and sets t = t_end exactly;
 *   - a sensor normaliser max|Q_alpha,k| equal to 0 gives s_hat_k = 0;
 *   - outflow is an edge-replicated ghost cell: streaming sources, central
 *     differences and the box filter clamp their neighbour index;
 *   - with retarget_every = K > 1 a retarget is forced when s_max > c;
 *   - the Ducros ratio (Eq. 33) takes dilatation and vorticity in lattice
 *     units (dt = dx/c times their central differences), so that its
 *     regulariser eps_theta is dimensionless.
 */
#ifndef VLBM_H
#define VLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vlbm_ctx vlbm_ctx;

typedef enum {
    VLBM_OK = 0,
    VLBM_EINVAL = -1,          /* invalid argument or configuration */
    VLBM_ENOMEM = -2,          /* device allocation failed */
    VLBM_EDEVICE = -3,         /* HIP runtime error */
    VLBM_ENONHYPERBOLIC = -4,  /* rho <= 0, c_s^2 <= 0 or 1 - b rho <= 0 (Eq. 14) */
    VLBM_ENONFINITE = -5,      /* NaN or Inf in the state */
    VLBM_EDONE = 1             /* nothing to do, not an error: t >= t_end already
                                  (vlbm_run_to_time) or t >= t_end_cap (vlbm_step) */
} vlbm_status;

/* Boundary kinds.  OUTFLOW: edge-replicated ghost cell (every neighbour index is
 * clamped into the grid).  PINNED (x edges only): the ghost cell holds a fixed
 * conserved state W_b at equilibrium, so the populations streaming in across
 * that edge are f^eq_i(W_b) at the current link speed (Eq. 20); the inflow edge
 * of the shock-vortex problem (Sec. IV.H).  The sensor's stencils treat a pinned
 * edge like an outflow edge. */
enum { VLBM_BC_PERIODIC = 0, VLBM_BC_OUTFLOW = 1, VLBM_BC_PINNED = 2 };
enum { VLBM_EOS_IDEAL = 0, VLBM_EOS_VDW = 1 };
enum { VLBM_SENSOR_OFF = 0, VLBM_SENSOR_A = 1, VLBM_SENSOR_B = 2, VLBM_SENSOR_AUTO = 3 };
/* precision of a context: FP64 populations and arithmetic; FP32 populations
 * and arithmetic; FP32 populations in HBM with FP64 arithmetic in registers */
enum { VLBM_FP64 = 0, VLBM_FP32 = 1, VLBM_FP32_MIXED = 2 };

/* Problem statement (Sec. II-III): lattice, grid, boundaries, EOS, time
 * stepping and sensor constants. */
typedef struct {
    int32_t dim;             /* 1 (D1Q2) or 2 (D2Q4) */
    int64_t nx, ny;          /* cells; ny == 1 when dim == 1; nx, ny >= 4 */
    double dx;               /* uniform spacing (dy == dx) */
    int32_t bc[4];           /* x-low, x-high, y-low, y-high: VLBM_BC_*; periodic must be set on both
                                sides of an axis; PINNED on x edges only */
    double bc_state[2][4];   /* W_b = (rho, rho u[, rho v], rho E) held at the x-low ([0]) and x-high
                                ([1]) edge when that edge is PINNED (physical energy gauge, first
                                dim + 2 entries used); it must be admissible (EINVAL otherwise) */
    int32_t eos;             /* VLBM_EOS_IDEAL: P = (gamma-1) rho e (Eq. 15); VLBM_EOS_VDW (Eqs. 16-17) */
    double gamma;            /* heat-capacity ratio; for vdW gamma = 1 + R/c_v */
    double vdw_a, vdw_b, vdw_R;
    double e_offset;         /* energy gauge of the stored populations: the energy component holds
                                rho E - e_offset rho.  The update is linear in W and in the flux Q
                                (Eqs. 20-22), so the shift is exact in real arithmetic; it keeps FP32
                                populations precise when e >> |u|^2 (dense gases).  Sensor, EOS and
                                every output (get_W, totals, get_f) use the physical gauge.  0 = off;
                                the adjoint entry points require 0. */
    double cfl;              /* target Courant number of the retargeting, c = s_max/CFL (Eq. 37) */
    int32_t retarget_every;  /* 1: every step; K > 1: every K steps (forced if s_max > c);
                                0: link speed frozen at c_fixed (no retarget, no landing) */
    double c_fixed;          /* link speed when retarget_every == 0 */
    int32_t sensor;          /* VLBM_SENSOR_*: OFF uses beta_const; A = Eq. 34; B = Eq. 35 */
    double beta_const, beta_min, beta_max, c_sensor;
    double eps_theta;        /* regulariser of the Ducros ratio (Eq. 33), dimensionless: dilatation and
                                vorticity enter in lattice units, dt = dx/c times their central
                                differences at the step's link speed, so beta is the same in any units
                                of length and time.  > 0; 1e-10 is the value the tests use */
    int32_t precision;       /* VLBM_FP64, VLBM_FP32 or VLBM_FP32_MIXED (populations and per-cell
                                arithmetic; clock, dt reduction and totals stay FP64) */
    void* stream;            /* hipStream_t, or NULL for the default stream */
} vlbm_config;

/* Validate a configuration without touching the device: VLBM_OK if
 * vlbm_create would accept it, VLBM_EINVAL otherwise (the same checks). */
vlbm_status vlbm_check_config(const vlbm_config* cfg);

/* Validate the configuration, allocate two population buffers, the clock and
 * reduction ring and scratch on the current device.  Ownership of *out passes
 * to the caller (release with vlbm_destroy).  EINVAL on a bad config, ENOMEM
 * on allocation failure. */
vlbm_status vlbm_create(const vlbm_config* cfg, vlbm_ctx** out);

/* Release every device allocation of the context (synchronises its stream). */
void vlbm_destroy(vlbm_ctx* ctx);

/* Initial state (Sec. III.E: the link speed is chosen from the initial data):
 * W0 (FP64, (dim+2, ny, nx)) is copied, c0 = s_max(W0)/CFL (or c_fixed),
 * populations f = f^eq(W0; c0) (Eq. 20), t = 0, n = 0.  ENONHYPERBOLIC /
 * ENONFINITE when W0 is not admissible. */
vlbm_status vlbm_init(vlbm_ctx* ctx, const double* W0, int32_t W0_on_device);

/* Advance exactly `nsteps` steps (fewer if t reaches t_end_cap, which then
 * lands exactly; pass INFINITY for no cap).  *steps_taken (nullable) receives
 * the steps executed.  VLBM_EDONE, with no step taken, when t >= t_end_cap
 * already.  On an EOS failure the state is left at the first inadmissible step
 * and ENONHYPERBOLIC / ENONFINITE is returned. */
vlbm_status vlbm_step(vlbm_ctx* ctx, int64_t nsteps, double t_end_cap, int64_t* steps_taken);

/* Advance until t == t_end exactly (Sec. III.E, final-step landing).
 * VLBM_EDONE, with no step taken, if t >= t_end already.
 *
 * Execution of vlbm_step and vlbm_run_to_time: the steps of a call are queued
 * without host synchronisation and the host reads the clock back once per
 * batch.  A D1Q2 grid of at most 2048 cells runs each batch of up to 4096
 * steps in one workgroup that keeps
 * the populations on chip between steps; the state
 * after the call, and every later call, is the same bit for bit as with one
 * launch per step (selected at creation with the environment variable
 * VLBM_D1_RESIDENT=0, for comparison). */
vlbm_status vlbm_run_to_time(vlbm_ctx* ctx, double t_end, int64_t* steps_taken);

/* out[dim+2] (host) = sum_x W(x) dx^dim in FP64, by a fixed-order tree
 * (deterministic).  Discrete conservation: Sec. III.A. */
vlbm_status vlbm_conserved_totals(vlbm_ctx* ctx, double* out);

/* W = sum_i f_i as FP64 (dim+2, ny, nx) into host or device memory. */
vlbm_status vlbm_get_W(vlbm_ctx* ctx, double* out, int32_t out_on_device);

/* beta(x) (Eqs. 34-35) of the current state: the field the next step uses,
 * FP64 (ny, nx) into host or device memory. */
vlbm_status vlbm_get_beta(vlbm_ctx* ctx, double* out, int32_t out_on_device);

/* Raw populations in the context's precision, (2*dim, dim+2, ny, nx) without
 * plane padding, into host or device memory. */
vlbm_status vlbm_get_f(vlbm_ctx* ctx, void* out, int32_t out_on_device);

/* Current time, link speed c and step count (synchronises). */
vlbm_status vlbm_get_clock(vlbm_ctx* ctx, double* t, double* c, int64_t* n);

/* Checkpoint / resume (no counterpart in the paper: a service of the library).
 * The state is the populations plus (t, c, n) and the reductions of the
 * current state, behind a 64-byte header naming the lattice, grid, precision
 * and plane layout of the context that saved it.  `buf` is a device buffer of
 * `bytes` >= vlbm_state_bytes() bytes, owned by the caller.  vlbm_restore
 * returns VLBM_EINVAL, leaving the context unchanged, when the buffer is too
 * small, when its header does not match the context or when its clock is not
 * valid.  Both synchronise the stream.  restore(save(x)) resumes bitwise. */
size_t vlbm_state_bytes(const vlbm_ctx* ctx);
vlbm_status vlbm_save(vlbm_ctx* ctx, void* buf, size_t bytes);
vlbm_status vlbm_restore(vlbm_ctx* ctx, const void* buf, size_t bytes);

/* Elements per population plane (padding included) and bytes of one
 * population array (2*dim*(dim+2) planes) in the context's precision; the
 * raw entry points below use this layout. */
int64_t vlbm_plane_elems(const vlbm_ctx* ctx);
size_t vlbm_population_bytes(const vlbm_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Raw, stream-ordered entry points for differentiation with the link speed
 * frozen at c_fixed (retarget_every must be 0).  All pointers are device
 * pointers.  A population array uses the padded plane layout above.  A `norms`
 * array (VLBM_NORMS_LEN doubles) describes the state it belongs to: 16 copies,
 * 16 doubles apart, of (s_max, then max_{x,alpha}|Q_alpha,k| for each component
 * k, Eq. 30); each quantity is the maximum over the copies (kernels spread
 * their atomic maxima over the copies).  The caller allocates it; raw_init and
 * raw_step overwrite their output array entirely.  The adjoint entry points
 * (raw_adjoint_step, raw_init_adjoint, raw_moments_adjoint) return EINVAL when
 * e_offset != 0 or an edge is PINNED.
 * ------------------------------------------------------------------------- */
#define VLBM_NORMS_LEN 256

/* f0 = f^eq(W0; c_fixed) (Eq. 20) and its norms.  W0: FP64 (dim+2, ny, nx). */
vlbm_status vlbm_raw_init(vlbm_ctx* ctx, const double* W0, void* f0, double* norms0);

/* One frozen-speed step f_out = step(f_in) (Eqs. 20-22, 28-35), reading the
 * sensor normalisers from norms_in and writing the norms of f_out.  f_in and
 * f_out start on 16-byte boundaries (the D1Q2 step reads and writes 16 bytes
 * per lane): VLBM_EINVAL otherwise. */
vlbm_status vlbm_raw_step(vlbm_ctx* ctx, const void* f_in, const double* norms_in, void* f_out,
                          double* norms_out);

/* Adjoint (vector-Jacobian product) of vlbm_raw_step at the state f_n with its
 * norms: lam_n = (d step / d f_n)^T lam_np1, including the EOS closure, the
 * sensor stencil and the max-normaliser (sub-gradient to the first arg-max in
 * (alpha, y, x) order); clip derivative 1 on (0,1) and 0 outside; the
 * derivative of the square root at 0 is taken as 0. */
vlbm_status vlbm_raw_adjoint_step(vlbm_ctx* ctx, const void* f_n, const double* norms_n,
                                  const void* lam_np1, void* lam_n);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): vlbm_raw_adjoint_step
 * with the per-wavefront records of the fused D2Q4 adjoint march (its only
 * scratch) in a static device array of 4096 records (384 KiB) instead of the
 * context's buffer.  It allocates nothing and calls no allocating routine; the
 * first call on a device looks up that device's copy of the array.  Same
 * arguments, result and stream ordering as vlbm_raw_adjoint_step, bit for bit.
 * VLBM_EINVAL for a context on the multi-pass adjoint (D1Q2, or
 * VLBM_ADJ_MULTIPASS set at creation) or a grid whose tiling needs more than
 * 4096 march records (strips of 56 columns times row segments), with the
 * counts in vlbm_last_error.  Every call on one GPU shares that GPU's array
 * and overwrites all of the records it reads, so nothing carries over between
 * calls; calls that overlap in time on one GPU (other streams, other threads)
 * race on it. */
vlbm_status vlbm_raw_adjoint_step_static(vlbm_ctx* ctx, const void* f_n, const double* norms_n,
                                         const void* lam_np1, void* lam_n);

/* Adjoint of vlbm_raw_init: W0bar (FP64 (dim+2, ny, nx), overwritten) =
 * (d f0/d W0)^T lam0 at the state W0. */
vlbm_status vlbm_raw_init_adjoint(vlbm_ctx* ctx, const double* W0, const void* lam0, double* W0bar);

/* W = sum_i f_i of a population array, FP64 (dim+2, ny, nx). */
vlbm_status vlbm_raw_moments(vlbm_ctx* ctx, const void* f, double* W);

/* Adjoint of vlbm_raw_moments: lam_i = Wbar for every direction i. */
vlbm_status vlbm_raw_moments_adjoint(vlbm_ctx* ctx, const double* Wbar, void* lam);

/* Message of the last failing call on this context (valid until the next call). */
const char* vlbm_last_error(const vlbm_ctx* ctx);

/* Measurement aid, not part of the method: the attainable-bandwidth references
 * that roofline fractions are read against.  mode 0 copies `bytes` (a multiple
 * of 16) from the device buffer src to the device buffer dst, which must not
 * overlap, with a grid-stride kernel of 16-byte non-temporal loads and stores.
 * mode 1 only reads src (four independent 16-byte loads in flight per lane)
 * and writes one 16-byte XOR of the words each workgroup read to dst:
 * vlbm_copy_probe_read_bytes(bytes) bytes (at most 128 KiB), which dst must
 * hold; the XOR of those words is the XOR of all 16-byte words of src.
 * Stream-ordered on `stream` (a hipStream_t; NULL: the null stream), returns
 * before the kernel completes; the caller owns both buffers.  VLBM_EINVAL for a
 * null pointer, a size that is not a multiple of 16 or an unknown mode,
 * VLBM_EDEVICE if the launch fails. */
vlbm_status vlbm_copy_probe(const void* src, void* dst, size_t bytes, void* stream, int32_t mode);
size_t vlbm_copy_probe_read_bytes(size_t bytes);

/* Measurement aid, not part of the method: `nlaunch` launches of a kernel with
 * the D2Q4 step's memory access pattern and none of its arithmetic (same grid,
 * tiling, halos, addressing and loads in flight; loads every population plane
 * of each row, stores the owned cells' values where the step stores its
 * post-collision populations), reading the current populations and writing the
 * context's spare population buffer, so the state is left as it was.  Its rate
 * bounds what the step's access pattern can move through HBM.  Stream-ordered,
 * no synchronisation.  VLBM_EINVAL for a D1Q2 or uninitialised context. */
vlbm_status vlbm_probe_march(vlbm_ctx* ctx, int32_t nlaunch);

#ifdef __cplusplus
}
#endif

#endif /* VLBM_H */
