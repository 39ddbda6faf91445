/*
 * ibmlbm.h - C ABI of the MI355X (gfx950) immersed-boundary lattice Boltzmann
 * solver: D3Q19 BGK with Guo forcing (Sec. 2.1, Eqs. 1-9) coupled to the
 * implicit velocity-correction immersed boundary method (Sec. 2.2,
 * Eqs. 10-19) on rigid elliptic foils in clap & fling motion (Sec. 3.3,
 * Eqs. 23-24) or on the figure-eight stroke (Sec. 3.2, Eqs. 20-22), with
 * force integration over the markers (Sec. 3.7, Eq. 26).  Faces take
 * periodic, bounce-back wall, equilibrium or Zou-He inflow/outflow rules
 * (Sec. 2.1, Sec. 3.1).  nz = 1 with a periodic span is the paper's 2D
 * D2Q9 scheme exactly (summing the D3Q19 populations of equal (c_x, c_y)
 * gives the D2Q9 weights of Eq. 5, equilibrium, forcing and streaming).
 *
 * Conventions (all calls):
 *  - Lattice units, dx = dt = 1.  The box has nx*ny*nz cells; host arrays are
 *    float64, x fastest, then y, then z; vector fields are three such planes
 *    (x-, y-, z-component).  Distributions use the canonical D3Q19 order
 *      0:(0,0,0) 1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1) 6:(0,0,-1)
 *      7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0) 11:(1,0,1) 12:(-1,0,-1)
 *      13:(1,0,-1) 14:(-1,0,1) 15:(0,1,1) 16:(0,-1,-1) 17:(0,1,-1) 18:(0,-1,1)
 *  - Every call returns an int status: 0 (IBMLBM_OK) or a negative code.  No
 *    exception crosses the ABI; ibmlbm_last_error() gives the message.
 *  - Device memory is owned by the caller: one workspace of at least
 *    ibmlbm_workspace_bytes() bytes, 256-byte aligned, handed to create().
 *    The library never allocates device memory.  The library owns only the
 *    host-side handle and, per handle, a small pinned host buffer (about
 *    150 KB) through which it uploads the launch arguments of 64 steps at a
 *    time.  Input arrays are copied, never retained.
 *  - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *    void*; NULL = the null stream).  step() only enqueues; forces(),
 *    fields(), mass() and destroy() synchronise the stream.  A device error
 *    raised by enqueued work is reported by the next synchronising call as
 *    IBMLBM_EDEVICE.
 *  - A handle is not thread-safe.  Distinct handles on distinct streams may
 *    be used concurrently from one thread or several.
 */
#ifndef IBMLBM_H
#define IBMLBM_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define IBMLBM_API __attribute__((visibility("default")))
#else
#define IBMLBM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibmlbm_s* ibmlbm_t;

enum {
  IBMLBM_OK = 0,
  IBMLBM_EINVAL = -1,    /* bad argument or configuration */
  IBMLBM_ENOMEM = -2,    /* workspace too small */
  IBMLBM_EDEVICE = -3,   /* HIP runtime or kernel error */
  IBMLBM_EDIVERGED = -4, /* a check step found a non-finite density (sticky) */
  IBMLBM_ESTATE = -5,    /* call out of order (e.g. fields before init) */
  IBMLBM_ERANGE = -6     /* requested history no longer (or not yet) held */
};

/* Face boundary kinds; faces are ordered -x, +x, -y, +y, -z, +z.
 * PERIODIC must be given on both faces of an axis.  The inflow/outflow
 * kinds are allowed on x faces only (Sec. 2.1: uniform-velocity inflow,
 * atmospheric-pressure outflow; walls by half-way bounce-back).
 * VELOCITY / PRESSURE: the populations entering through the face come from
 * a ghost layer at equilibrium with the prescribed velocity (density of the
 * boundary cell) or the prescribed density (velocity of the boundary cell).
 * ZH_VELOCITY / ZH_PRESSURE: the Zou-He scheme the paper names for its
 * cylinder case (Sec. 3.1, its ref. [21]): the entering populations of each
 * boundary cell are rebuilt from its known ones so that its density and
 * momentum take the prescribed velocity (density from the known
 * populations) or the prescribed density (transverse velocity zero), with
 * non-equilibrium bounce-back of the normal population and a transverse
 * momentum correction (D3Q19 form).  Boundary cells whose entering links
 * also touch a y or z wall keep the equilibrium ghost rule. */
enum {
  IBMLBM_BC_PERIODIC = 0, IBMLBM_BC_WALL = 1, IBMLBM_BC_VELOCITY = 2, IBMLBM_BC_PRESSURE = 3,
  IBMLBM_BC_ZH_VELOCITY = 4, IBMLBM_BC_ZH_PRESSURE = 5
};

/* Storage of the distributions.  FP32 stores f_i - w_i in float; the
 * FP16/BF16 forms store f_i - w_i in 16 bits.  Collision arithmetic is FP32
 * in every form. */
enum { IBMLBM_FP32 = 0, IBMLBM_FP16_DEV = 1, IBMLBM_BF16_DEV = 2 };

/* alpha(t) of a foil: CONST = alpha_mean; SIN = alpha_mean + alpha_amp
 * sin(2 pi t / T + phase) (Eq. 21, Eq. 23 as printed); ABS_SIN =
 * alpha_mean + alpha_amp |sin(2 pi t / T + phase)| (Eq. 23 read with the
 * text's 0..60 degree range). */
enum { IBMLBM_ALPHA_CONST = 0, IBMLBM_ALPHA_SIN = 1, IBMLBM_ALPHA_ABS_SIN = 2 };

enum { IBMLBM_FIELD_RHO = 0, IBMLBM_FIELD_U = 1, IBMLBM_FIELD_FDIST = 2 };

/* Marker-level outputs of the last step (see ibmlbm_markers). */
enum { IBMLBM_MARKER_X = 0, IBMLBM_MARKER_U = 1, IBMLBM_MARKER_RHS = 2,
       IBMLBM_MARKER_DU = 3, IBMLBM_MARKER_RHO = 4, IBMLBM_MARKER_DA = 5 };

typedef struct {
  int32_t nx, ny, nz;     /* cells, each >= 4; x is the free-stream axis */
  int32_t bc[6];          /* -x,+x,-y,+y,-z,+z (IBMLBM_BC_*) */
  double  tau;            /* BGK relaxation time, Eq. 3: tau = 3 nu + 1/2 > 1/2 */
  double  u_in[3];        /* velocity of VELOCITY faces */
  double  rho_out;        /* density of PRESSURE faces (1 = atmospheric) */
  double  body_force[3];  /* uniform force density added to F (tests) */
  int32_t storage;        /* IBMLBM_FP32 / FP16_DEV / BF16_DEV */
  int32_t check_interval; /* every k-th step records the FP64 mass and a
                             non-finite check; 0 = never */
  double  u_ref;          /* coefficients: C = F / (0.5 u_ref^2 area_ref) */
  double  area_ref;
  int64_t history_steps;  /* capacity of the device force-history ring, >= 1 */
} ibmlbm_config;

/* One rigid elliptic foil (Sec. 3.2-3.3) extruded over the whole periodic
 * span (z), one marker layer per lattice plane at z = k + 1/2. */
typedef struct {
  double  chord, thickness;  /* ellipse axes; aspect ratio = chord/thickness */
  double  ds;                /* target marker spacing along the perimeter (1.0) */
  double  hinge[2];          /* pivot (x, y) at the reference time */
  double  pivot_frac;        /* pivot on the chord: 0 = LE, 0.5 = centre, 1 = TE */
  double  theta0;            /* chord angle at alpha = 0 (LE points to -x at 0) */
  double  sense;             /* +1 or -1: theta = theta0 + sense * alpha(t);
                                lift is counted along -sense * y */
  int32_t alpha_shape;       /* IBMLBM_ALPHA_* */
  int32_t pad_;
  double  alpha_mean, alpha_amp, period_steps, phase;
  double  trans_amp, trans_angle;  /* Eq. 20: pivot moves trans_amp cos(2 pi t/T +
                                      phase) along angle trans_angle */
} ibmlbm_wing;

/* Bytes of device workspace needed for cfg and the given foils (n_wings may
 * be 0).  Returns 0 if the configuration is invalid (among the limits:
 * nx, ny >= 4; nx ny nz <= 2^34 cells; ny nz < 2^31 lattice rows;
 * nx < 2^24). */
IBMLBM_API size_t ibmlbm_workspace_bytes(const ibmlbm_config* cfg, int32_t n_wings,
                              const ibmlbm_wing* wings);

/* Validate cfg and bind a handle to the caller's device workspace and stream.
 * Lattice storage is carved from the start of the workspace; set_kinematics
 * carves the marker storage from the rest.  The fields start undefined:
 * call ibmlbm_init_fields before stepping.  EINVAL for a bad config, ENOMEM
 * if bytes is below the lattice part of ibmlbm_workspace_bytes. */
IBMLBM_API int ibmlbm_create(const ibmlbm_config* cfg, void* dev_workspace, size_t bytes,
                  void* hip_stream, ibmlbm_t* out);

/* Set the state to the equilibrium (Eq. 4) of rho (N values, NULL = 1) and u
 * (3N values, NULL = 0), or, if fdist (19N values) is given, to those
 * post-collision distributions (exact resume of a state read with
 * IBMLBM_FIELD_FDIST).  Resets the step counter to step0. */
IBMLBM_API int ibmlbm_init_fields(ibmlbm_t h, const double* rho, const double* u,
                       const double* fdist, int64_t step0);

/* ibmlbm_create for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * dev_state (256-byte aligned, caller-owned) holds only the two lattice
 * states; bytes >= ibmlbm_workspace_bytes(cfg, 0, NULL) is enough.  Every
 * other region of the solve (launch arguments, mass partials and flags,
 * marker data, node-box images, the force-history ring) lives in a static
 * device array of the library, 64 MiB per device, held from the first such
 * call on a device until the process ends; no pinned host buffer is made and
 * nothing is allocated with hipMalloc, hipHostMalloc or any other allocator.
 * The device current at the call must be the stream's.  All handles made
 * this way on one device share that array and keep its last contents:
 * create and set_kinematics clear what must start at zero, and two such
 * handles used at the same time on one device race.  ENOMEM (message naming
 * the limit) when the lattice's regions, or the markers' at
 * set_kinematics, exceed the array; other errors as ibmlbm_create. */
IBMLBM_API int ibmlbm_create_noalloc(const ibmlbm_config* cfg, void* dev_state, size_t bytes,
                                     void* hip_stream, ibmlbm_t* out);

/* Place the markers of n_wings foils (n_wings = 0 removes them).  Each
 * foil's perimeter gets round(P/ds) markers at equal arc length; the
 * surface element is P/round(P/ds) x 1.  EINVAL if a marker support could
 * leave the box on a non-periodic axis, if the span is not periodic, if
 * two foils' supports could overlap during the motion, if a foil's
 * perimeter system (Eq. 18) is numerically singular, or if the span has more
 * layers than one marker's interpolation block holds in local memory (the
 * message names the limit, about 425 layers).  ENOMEM if the workspace
 * cannot hold the markers. */
IBMLBM_API int ibmlbm_set_kinematics(ibmlbm_t h, int32_t n_wings, const ibmlbm_wing* wings);

/* Enqueue n time steps (Sec. 2.2): streaming, moments, marker kinematics at
 * t = step, interpolation, the no-slip solve A X = B (Eq. 19, minimum-norm
 * solution), spreading, Guo-forced collision and force integration. */
IBMLBM_API int ibmlbm_step(ibmlbm_t h, int32_t n);

/* Enqueue n time steps of each of n_handles solves (1..64 distinct,
 * initialised handles bound to one stream), in lock step: each stage of a
 * step is one grouped launch over all handles that use the same kernel
 * (same storage, with or without foils, body force, check step), so many
 * small solves share the device the way one large solve does.  This is how
 * the parametric sweep of Sec. 3.3-3.5 (Re, J and f varied) is served.
 * Every solve runs the same kernels with the same arguments as under
 * ibmlbm_step, so its results do not depend on the other solves of the
 * batch.  Timing events (ibmlbm_timing) bracket single-handle steps
 * only.  EINVAL for a bad handle list or mixed streams; ESTATE if a handle
 * is not initialised. */
IBMLBM_API int ibmlbm_step_batch(ibmlbm_t* hs, int32_t n_handles, int32_t n);

/* Move the handle to another HIP stream: waits for the work enqueued on
 * its current stream, then enqueues everything after on hip_stream.  A
 * server prepares a new solve (create, set_kinematics, init_fields, which
 * synchronise their stream) on a side stream while other solves keep
 * running, then moves it to the stream of its batch (ibmlbm_step_batch). */
IBMLBM_API int ibmlbm_set_stream(ibmlbm_t h, void* hip_stream);

/* Number of steps taken since init_fields (plus step0). */
IBMLBM_API int64_t ibmlbm_step_count(ibmlbm_t h);

/* Copy force history rows [first, first+count) to out[count][n_wings][8]
 * (host memory, caller-owned, row-major), the force integration of Sec. 3.7:
 * the Lagrangian force density f_B = 2 rho_B du_B / dt of each marker (Eq. 26)
 * times its surface element, summed over the foil, with the sign turned to
 * give the force on the body; then
 *   Fx, Fy, Fz  force on the body,
 *   Mz          its moment about the foil's pivot, sum (X - X_pivot) x f,
 *   CL          lift = lateral force, counted along -sense * y (outward for a
 *               mirrored pair), over 0.5 u_ref^2 area_ref (Sec. 3.6),
 *   CT, CD      thrust -Fx and drag Fx over the same,
 *   CM          Mz over 0.5 u_ref^2 area_ref chord.
 * Synchronises the stream.  ERANGE if a row is not in the ring, ESTATE with
 * no foils, EDIVERGED if a check step saw a non-finite density or a perimeter
 * system became singular, EDEVICE if a foil's support nodes outnumbered the
 * band-moment grid the host sized for them (the rows are still copied). */
IBMLBM_API int ibmlbm_forces(ibmlbm_t h, int64_t first, int64_t count, double* out);

/* Copy a field of the current state to host float64 (caller-owned, x
 * fastest): RHO (N: rho = sum_i f_i, Eq. 2), U (3N: the velocity
 * u* = (sum_i c_i f_i + F_body/2)/rho of Eqs. 2, 9 and 11, of the streamed
 * distributions the next step starts from, before its IBM correction),
 * FDIST (19N: the post-collision state f* of Eq. 7, canonical order).
 * Synchronises the stream; RHO and U use the other state buffer as scratch.
 * ESTATE before init_fields, EINVAL for an unknown field. */
IBMLBM_API int ibmlbm_fields(ibmlbm_t h, int32_t which, double* out);

/* Marker data of the last completed step, float64, marker order
 * wing-major, then perimeter, then span layer: X, U, RHS (B of Eq. 19) and
 * DU (du_B) are 3 per marker, RHO and DA one per marker. */
IBMLBM_API int ibmlbm_markers(ibmlbm_t h, int32_t which, double* out);
IBMLBM_API int32_t ibmlbm_marker_count(ibmlbm_t h);

/* Last FP64 mass check (sum of rho over all cells) and its step; *step = -1
 * if none yet.  Returns EDIVERGED once a check has seen a non-finite value. */
IBMLBM_API int ibmlbm_mass(ibmlbm_t h, int64_t* step, double* mass);

/* Kernel timing: with enable = k > 0 the collide-stream launch and the
 * marker kernels of every k-th step are bracketed by HIP events (recorded
 * without a system-scope fence) on the handle's stream; read_timing
 * synchronises, returns the summed milliseconds, count and updated cells of
 * the bracketed collide launches and the summed marker milliseconds, and
 * resets the sums.  enable = 0 stops recording. */
IBMLBM_API int ibmlbm_timing(ibmlbm_t h, int32_t enable);
IBMLBM_API int ibmlbm_read_timing(ibmlbm_t h, double* collide_ms, int64_t* collide_launches,
                                  double* collide_cells, double* marker_ms);

/* Algorithmic HBM bytes of one collide-stream cell update for this handle's
 * storage (19 reads + 19 writes of one stored value). */
IBMLBM_API int32_t ibmlbm_bytes_per_cell(ibmlbm_t h);

/* Synchronise and release the handle (not the workspace). */
IBMLBM_API int ibmlbm_destroy(ibmlbm_t h);

/* Message of the last failed call on h (thread-local when h is NULL). */
IBMLBM_API const char* ibmlbm_last_error(ibmlbm_t h);

/* Clap & fling physics to lattice units (Eq. 3, Eq. 22, Eq. 24; Sec. 3.4):
 * U_tip = kappa f, nu = U_tip chord / Re, tau = 3 nu + 1/2, U_inf = J U_tip,
 * period T = 2 Phi chord / U_tip with Phi = 120 degrees. */
IBMLBM_API int ibmlbm_lattice_params(double Re, double J, double f, double chord, double kappa,
                          double* tau, double* u_inf, double* u_tip, double* period_steps);

/* Fixed foil in a uniform stream (a plate at an angle of attack, Sec. 3.2-3.3
 * setups; the cylinder of Sec. 3.1): Re = u_inf chord / nu, so
 * nu = u_inf chord / Re and tau = 3 nu + 1/2 (Eq. 3 in lattice units).  EINVAL
 * unless Re, u_inf and chord are > 0. */
IBMLBM_API int ibmlbm_plate_params(double Re, double u_inf, double chord, double* tau);

/* Figure-eight hovering stroke (Sec. 3.2, Eqs. 20-22): Re = U_tip c / nu with
 * the largest speed of the wing centre U_tip = pi f A0 (Eq. 22).  Given the
 * lattice tip speed u_tip: nu = u_tip chord / Re, tau = 3 nu + 1/2 (Eq. 3) and
 * the period 1/f = pi A0 / u_tip steps.  EINVAL unless every input is > 0. */
IBMLBM_API int ibmlbm_figure_eight_params(double Re, double u_tip, double chord, double a0,
                                          double* tau, double* period_steps);

#ifdef __cplusplus
}
#endif
#endif /* IBMLBM_H */
