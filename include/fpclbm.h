/*
 * fpclbm.h - C ABI of the MI355X (gfx950) implementation of the Fokker-Planck
 * central-moment double-distribution lattice Boltzmann method for thermal
 * convection (Schupbach & Premnath, arXiv 2504.09041).
 *
 * One time step n advances every lattice node by the fused update
 *   pull-stream with wall rules  (Eq. LBMsteps-stream / LBMsteps-streamg, Sec. 6.1)
 *   -> macros rho, u, T and the Boussinesq force   (App. A Step 7, Sec. 6.1)
 *   -> fluid collision: central moments, relaxation toward the Fokker-Planck
 *      attractors with renormalised diffusion tensor above second order and
 *      body-force sources                          (Sec. 4.1-4.2, 5.1-5.2, App. A)
 *   -> thermal collision with option-A attractors   (Sec. 4.3-4.4, 5.3, App. B/C;
 *      option B and the Maxwellian comparator of Sec. 7 are selectable)
 *   -> store the post-collision populations (64-node tiles, see fpc_state_bytes).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every function returns an int status: FPC_OK (0) or a negative FPC_ERR_*
 *   code.  Nothing throws across the ABI.  After an error, fpc_last_error()
 *   returns a message (thread-local, valid until the next call on that thread).
 * - Arguments are validated on the host before any launch; a call that fails
 *   validation has no side effect.
 * - "device pointer" means memory on the GPU the simulation runs on
 *   (e.g. a torch CUDA tensor's data_ptr); "host pointer" means CPU memory.
 * - Grid: node (i, j, k), x fastest; nz = 1 in 2D.  N = nx * ny * nz.
 *   Walls lie halfway between the outermost node and its missing neighbour.
 * - Faces are indexed -x, +x, -y, +y, -z, +z (FPC_FACE_*).
 * - All calls that launch work are asynchronous on the simulation's stream,
 *   except those documented as synchronising.
 * - The caller owns the two state buffers and the stream; the library owns
 *   only small scratch buffers (reductions) freed by fpc_destroy.
 */
#ifndef FPCLBM_H
#define FPCLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define FPC_OK 0
#define FPC_ERR_ARG (-1)      /* invalid argument (null pointer, bad enum, rate outside (0,2), ...) */
#define FPC_ERR_SIZE (-2)     /* sizes out of range or inconsistent */
#define FPC_ERR_HIP (-3)      /* a HIP runtime call failed; message in fpc_last_error() */
#define FPC_ERR_UNSTABLE (-4) /* diagnostics found NaN/Inf or |u| above the watchdog limit */
#define FPC_ERR_STATE (-5)    /* the call does not fit the simulation's configuration */

/* Lattice pairs (fluid + thermal). */
#define FPC_D2Q9_D2Q5 1   /* D2Q9 fluid (Eqs. ex, ey) + D2Q5 thermal (axis subset of D2Q9) */
#define FPC_D3Q27_D3Q7 2  /* D3Q27 fluid (Sec. 5.2) + D3Q7 thermal (axis subset of D3Q27) */
#define FPC_D2Q9_D2Q9 3   /* D2Q9 fluid + the paper's D2Q9 thermal lattice (Sec. 4.4, App. B) */
#define FPC_D3Q27_D3Q15 4 /* D3Q27 fluid + the paper's D3Q15 thermal lattice (Sec. 5.4, App. C) */

/* Collision models (fpc_params.model). */
#define FPC_MODEL_FP 0  /* Fokker-Planck central-moment attractors (the method) */
#define FPC_MODEL_MCM 1 /* Maxwellian central-moment attractors: the comparator of Sec. 7 */

/* Thermal attractors above second order (fpc_params.thermal_option; D2Q9 / D3Q15 thermal only). */
#define FPC_THERMAL_OPTION_A 0 /* diffusion tensor c^_s^2 I at every order (Eq. Dij2D_goptionA) */
#define FPC_THERMAL_OPTION_B 1 /* renormalised by the post-collision second order over T (Eq. Dij2D_g) */

/* Storage precision of the populations. */
#define FPC_FP64 0     /* populations f, g stored and collided in FP64 */
#define FPC_FP32_DEV 1 /* FP32 deviations f - w rho0 and g - w^T Tr (Tr: T_ref_slope/axis), collided in FP32 */

/* Face kinds (fluid rule + thermal rule). */
#define FPC_BC_PERIODIC 0          /* must be set on both faces of an axis */
#define FPC_BC_NOSLIP_ADIABATIC 1  /* halfway bounce-back for f and g */
#define FPC_BC_NOSLIP_DIRICHLET 2  /* bounce-back for f, anti-bounce-back for g at wall_T */
#define FPC_BC_LID_ADIABATIC 3     /* moving-wall bounce-back (lid_u) for f, bounce-back for g */
#define FPC_BC_LID_DIRICHLET 4     /* moving-wall bounce-back for f, anti-bounce-back for g */

/* fpc_params.T_ref_axis: pick the FP32 storage reference from the walls. */
#define FPC_TREF_AUTO (-2)

#define FPC_FACE_XM 0
#define FPC_FACE_XP 1
#define FPC_FACE_YM 2
#define FPC_FACE_YP 3
#define FPC_FACE_ZM 4
#define FPC_FACE_ZP 5

/*
 * Simulation parameters.  Fill with fpc_params_default(), then one of the
 * fpc_params_natural() / fpc_params_mixed() helpers or by hand.
 *
 * omega_f: fluid rates, one per central moment in the paper's order, with the
 *   diagonal second-order slots holding the rates of their combinations:
 *   2D (App. A Step 3): w0..w8 <-> (00, 10, 01, 20+02, 20-02, 11, 21, 12, 22).
 *   3D: (000, 100, 010, 001, 110, 101, 011, 200+020+002, 200-020, 200-002,
 *        120, 102, 210, 012, 201, 021, 111, 220, 202, 022, 211, 121, 112,
 *        122, 212, 221, 222)  (moment order of Sec. 5.2).
 *   Slot 0 has no effect (mass is conserved).
 * omega_g: thermal rates.  D2Q5 (App. B Step 3): (00, 10, 01, 20+02, 20-02);
 *   D3Q7 (App. C Step 3): (000, 100, 010, 001, 200, 020, 002);
 *   D2Q9 (App. B Step 3): (00, 10, 01, 20+02, 20-02, 11, 21, 12, 22);
 *   D3Q15 (App. C Step 3): (000, 100, 010, 001, 110, 101, 011, 200, 020, 002,
 *          120, 012, 201, 111, 220).
 * Every rate in use must lie in (0, 2).
 */
typedef struct fpc_params {
  int lattice;   /* FPC_D2Q9_D2Q5, FPC_D3Q27_D3Q7, FPC_D2Q9_D2Q9 or FPC_D3Q27_D3Q15 */
  int precision; /* FPC_FP64 or FPC_FP32_DEV */
  int nx, ny, nz;
  double omega_f[27];
  double omega_g[15];
  double cs2_T;  /* thermal diffusion parameter c^_s^2; default 1/3 (D2Q5, D2Q9, D3Q15), 1/4 (D3Q7) */
  double g_beta; /* buoyancy per unit temperature: F = g_beta (T - T0) along up_axis */
  double T0;     /* Boussinesq reference temperature; also the FP32-deviation offset of g */
  double rho0;   /* reference density: initial density, moving-wall density, FP32-deviation offset of f */
  double dT_ref; /* temperature difference used to scale the Nusselt number */
  int up_axis;   /* 0, 1, 2: axis along which buoyancy acts (y in 2D, z in 3D typically) */
  int bc[6];     /* FPC_BC_* per face */
  double wall_T[6];   /* Dirichlet wall temperature per face (uniform) */
  double lid_u[6][3]; /* wall velocity per face (lid faces only; must be tangential) */
  /* Optional per-node Dirichlet temperature on a face (device pointer, FP64, or NULL).
   * Layout: the face's two tangential axes, slower first (e.g. -y face in 3D: [z][x];
   * in 2D a -y face profile has nx values).  Read on every step, so it can be changed
   * between steps; the library never frees it. */
  const double* wall_T_profile[6];
  /* FP32-deviation storage reference of g (ignored for FPC_FP64).  The stored
   * thermal values are g - w^T Tr(x), with Tr one of:
   *   T_ref_axis = FPC_TREF_AUTO (the default of fpc_params_default): the
   *     conduction profile between the pair of Dirichlet faces (FPC_BC_*_DIRICHLET
   *     on both faces of an axis) with the largest wall-temperature difference,
   *     Tr(x) = T0 + s (x_k - (n_k - 1) / 2) with s = (wall_T[+k] - wall_T[-k]) / n_k
   *     (walls halfway outside the outermost nodes); the uniform T0 if there is
   *     no such pair.  fpc_storage_reference() reports the choice.
   *   T_ref_axis = k >= 0: the affine profile Tr(x) = T0 + T_ref_slope (x_k - (n_k - 1) / 2)
   *     (fpc_params_conduction_reference() fills it for a chosen axis); axis k
   *     must not be periodic and the slope must be finite.
   *   T_ref_axis = -1: the uniform reference T0 (the literal g - w^T T0 form).
   * An affine reference changes only what is stored: the algorithm computed is
   * the same.  Between two Dirichlet walls it keeps the stored values to the
   * departure from conduction, which keeps FP32 rounding in the wall layers
   * (and the wall Nusselt number) far below that of the uniform form. */
  double T_ref_slope;
  int T_ref_axis;
  /* Collision model, FPC_MODEL_FP (default) or FPC_MODEL_MCM.  The MCM
   * comparator replaces every attractor by the Maxwellian central moment
   * (rho or T times prod c(m_d), c(0) = 1, c(1) = 0, c(2) = c_s^2 or c^_s^2):
   * on D2Q5 / D3Q7 thermal it differs from FP in the fluid orders >= 4 only. */
  int model;
  /* FPC_THERMAL_OPTION_A (default) or _B; only the D2Q9 / D3Q15 thermal
   * lattices have moments above second order for it to act on. */
  int thermal_option;
} fpc_params;

typedef struct fpc_sim fpc_sim;

/* sizeof(fpc_params) as compiled into the library: lets a binding check its
 * copy of the struct layout before the first call. */
size_t fpc_params_bytes(void);

/* Library version (major*10000 + minor*100 + patch). */
int fpc_version(void);

/* Message of the last error on the calling thread ("" if none). */
const char* fpc_last_error(void);

/* Zero *p, set lattice/precision/sizes, every rate to 1, cs2_T to the lattice
 * default, rho0 = 1, dT_ref = 1, T0 = 0, up_axis = 1 (2D) or 2 (3D), all faces
 * periodic, T_ref_axis = FPC_TREF_AUTO.  Fails with FPC_ERR_ARG / FPC_ERR_SIZE
 * on a bad lattice or size. */
int fpc_params_default(fpc_params* p, int lattice, int precision, int nx, int ny, int nz);

/*
 * Natural convection (Sec. 6.1): from Ra = g beta dT L^3 / (nu alpha), Pr = nu / alpha
 * and the force scale U0^2 / L = g beta dT, sets nu = U0 L sqrt(Pr / Ra),
 * alpha = nu / Pr, g_beta = U0^2 / (L dT), the shear rates from
 * nu = c_s^2 (1/w - 1/2) (Eq. transportcoeff2DFPCLBM, c_s^2 = 1/3) and the
 * first-order thermal rates from alpha = c^_s^2 (1/w - 1/2)
 * (Eq. thermaltransportcoeff2DFPCLBM).  Every other rate is set to 1.
 * L = number of nodes along L_axis; dT = T_hot - T_cold (stored in dT_ref);
 * T0 = (T_hot + T_cold) / 2.  Leaves bc/wall_T/lid_u untouched.
 */
int fpc_params_natural(fpc_params* p, double Ra, double Pr, double U0, int L_axis, double T_hot,
                       double T_cold);

/* Mixed convection (Sec. 7): nu = U L / Re, alpha = U L / Pe, g_beta = Ri U^2 / (L dT),
 * rates as in fpc_params_natural. */
int fpc_params_mixed(fpc_params* p, double Re, double Ri, double Pe, double U_lid, int L_axis,
                     double T_hot, double T_cold);

/* Set the FP32 storage reference to the conduction profile between the two
 * Dirichlet faces of `axis` (T_ref_axis = axis, T_ref_slope =
 * (wall_T[2 axis + 1] - wall_T[2 axis]) / n_axis, the linear profile through the
 * wall temperatures with the walls halfway outside the outermost nodes,
 * Sec. 6.1).  Call after the faces are set.  FPC_ERR_ARG if either face of the
 * axis is not a Dirichlet face or the axis is out of range. */
int fpc_params_conduction_reference(fpc_params* p, int axis);

/* The FP32 storage reference the parameters select (after FPC_TREF_AUTO is
 * resolved): *axis = k and *slope = s of Tr(x) = T0 + s (x_k - (n_k - 1) / 2),
 * or *axis = -1, *slope = 0 for the uniform T0 (always so for FPC_FP64).
 * Validates the parameters first (errors as fpc_state_bytes). */
int fpc_storage_reference(const fpc_params* p, int* axis, double* slope);

/* Bytes each of the two state buffers must hold, and the padded row length
 * nxp (nx rounded up to a multiple of 64).  State layout (elements of FP64
 * for FPC_FP64, FP32 for FPC_FP32_DEV): node (x, y, z) has the padded index
 * n = (z ny + y) nxp + x; nodes form tiles of 64 consecutive padded indices,
 * and tile t = n / 64 stores its Q = Qf + Qg populations (fluid 0..Qf-1, then
 * thermal) one after the other as runs of 64 values, so population q of node
 * n is element (t Q + q) 64 + n % 64.  Elements of padding nodes
 * (x >= nx) are never read or written by the step kernels.
 * bytes_per_buffer = nxp ny nz Q sizeof(element).
 * Validates the parameters first: FPC_ERR_ARG for invalid rates, faces, lid
 * velocities, references or codes; FPC_ERR_SIZE when an axis length is not
 * positive, a walled axis has fewer than 2 nodes, the padded node count
 * nxp ny nz reaches 2^31, or a state would hold more than 4e10 populations.
 * Either output pointer may be NULL. */
int fpc_state_bytes(const fpc_params* p, size_t* bytes_per_buffer, size_t* row_stride);

/*
 * Create a simulation that borrows two device buffers of at least
 * fpc_state_bytes() bytes each (256-byte aligned) and a hipStream_t (may be
 * NULL for the null stream).  Parameters are copied and validated.  Allocates
 * only reduction scratch: a few KiB, the wall-Nusselt slots (two doubles per
 * wall row of each tile) and the per-tile partials of fpc_step_diagnostics
 * (four doubles per 64-node tile, 0.5 B per node).  *out is set on success.
 */
int fpc_create(const fpc_params* p, void* bufA, void* bufB, void* hip_stream, fpc_sim** out);

/* Free the library-owned scratch and the handle (not the caller's buffers). */
int fpc_destroy(fpc_sim* s);

/* Change the stream later calls launch on. */
int fpc_set_stream(fpc_sim* s, void* hip_stream);

/*
 * Initial state: pre-collision f = w rho0, g = w^T T_init(x) (fluid at rest),
 * then one collision at every node (force from T_init), stored as S_0.
 * T_init: device pointer to N FP64 values [z][y][x].  Resets the step counter.
 */
int fpc_init(fpc_sim* s, const double* T_init);

/*
 * Advance nsteps >= 0 time steps (fused pull-stream-collide, Eq.
 * LBMsteps-stream / LBMsteps-streamg with the collision of Sec. 4-5),
 * asynchronously.  Small grids (at most 16 blocks of 256 nodes; any lattice
 * pair in 2D, or in 3D with FP32 storage; standard rate set)
 * advance up to 1024 steps per cooperative launch, with a grid-wide barrier
 * between steps, when the device supports cooperative launches; otherwise,
 * and on every other grid, one launch per step.  Both paths compute the
 * same step; they are compiled separately, so their states agree to rounding
 * (multiply-adds may be fused differently), not bit for bit.  A barrier that
 * times out (it cannot on a working device) leaves the state invalid and is
 * reported by the next fpc_diagnostics as FPC_ERR_HIP, after which the sim
 * uses per-step launches only.
 */
int fpc_step(fpc_sim* s, int nsteps);

/*
 * Allow (enable = 1, the default) or forbid (0) fpc_step's single-launch
 * multi-step path on small grids.  Errors: FPC_ERR_ARG (NULL, enable not 0/1).
 */
int fpc_set_multistep(fpc_sim* s, int enable);

/*
 * Polls a barrier wait of the multi-step path may repeat before it gives up
 * and raises the error flag (default 2^22, about a second; 0: give up at the
 * first unmet check).  A small value exercises the failure path from the
 * host: the waits end early, every block leaves its launch, and the next
 * fpc_diagnostics reports FPC_ERR_HIP (the state is then invalid and the path
 * off for this sim).  Errors: FPC_ERR_ARG (NULL).
 */
int fpc_set_multistep_wait_limit(fpc_sim* s, unsigned polls);

/* Number of multi-step (cooperative) launches fpc_step has made on this sim. */
int fpc_multistep_launches(const fpc_sim* s, long long* launches);

/*
 * Advance nsteps >= 0 time steps exactly as fpc_step, and after each step n
 * add weight * <Nu>_face(n) to acc[0]: the mean wall Nusselt number of
 * fpc_diagnostics on wall_face at the new time level n (Sec. 6.1 stencil
 * dT/dn = -8/3 T_w + 3 T(1/2) - 1/3 T(3/2), Nu = -(L / dT_ref) dT/dn).
 * acc: device pointer to one FP64 value, accumulated into (never
 * overwritten), so a time-averaged objective sum_n w <Nu>(n) builds up over
 * several calls without a host synchronisation.  The step kernel itself
 * forms the sums from the two wall layers of the state it writes (per-tile
 * partial sums in library-owned scratch, reduced in a fixed order into acc at
 * the end of the call), so a step costs about what fpc_step costs.
 * Asynchronous.  Errors: FPC_ERR_ARG (NULL, nsteps < 0, wall_face outside
 * 0..5, weight not finite), FPC_ERR_STATE (periodic face, or a z face in 2D).
 */
int fpc_step_nusselt(fpc_sim* s, int nsteps, int wall_face, double weight, double* acc);

/*
 * Advance nsteps >= 1 time steps as fpc_step and return the diagnostics of
 * the new time level without a separate pass over the state: the kernel of
 * the last step forms, after its stores, each node's FP64 macros from the
 * values it stores, exactly as fpc_diagnostics forms them from the stored
 * state (rho = rho_r + sum f, T = T_r + sum g, rho u = sum f e - F/2), and
 * reduces them over its 64-node tile; two small kernels then reduce the
 * tiles in a fixed order.  Writes out[0..4] = (mean wall Nusselt number on
 * wall_face by the fused accumulation of fpc_step_nusselt, or 0 for
 * wall_face = -1; KE; sum T; max |u|; number of nodes with a non-finite
 * macro), the layout of fpc_diagnostics_noalloc, to `out` (device pointer,
 * 5 FP64 values).  The values equal those fpc_diagnostics returns at the new
 * time level up to the order of the FP64 sums (relative differences of a few
 * ulps of the sum).  Asynchronous: no host synchronisation, and the watchdog
 * (out[4] != 0 or out[3] > 0.5) is left to the caller.  Uses the per-tile
 * partials allocated by fpc_create and the library's reduction scratch, so
 * calls on one sim are ordered by its stream.  Errors: FPC_ERR_ARG (NULL,
 * nsteps < 1, wall_face outside -1..5), FPC_ERR_STATE (periodic face, or a z
 * face in 2D), FPC_ERR_HIP (launch failure).
 */
int fpc_step_diagnostics(fpc_sim* s, int nsteps, int wall_face, double* out);

/*
 * One time step from a caller-owned state into another caller-owned state:
 * S_dst = Phi(S_src) (the fused pull-stream-collide of fpc_step), with this
 * simulation's parameters.  src, dst: device pointers, 256-byte aligned, each
 * of fpc_state_bytes() bytes in the storage layout (as written by fpc_save).
 * They must not overlap.  The simulation's own buffers and step counter are
 * untouched; asynchronous on the simulation's stream.  Lets a reverse sweep
 * rebuild the states of a checkpoint segment in place, without copies.
 */
int fpc_step_from(fpc_sim* s, const void* src, void* dst);

/* Steps taken since the last fpc_init / fpc_load. */
int fpc_get_step(const fpc_sim* s, long long* step);

/*
 * Macros of the current time level n (from the stored post-collision state:
 * rho = sum f, T = sum g, rho u = sum f e - F/2, equal to the pre-collision
 * values by conservation).  Device pointers to N FP64 values each, u holds
 * d planes [x-comp][N], [y-comp][N] (, [z-comp][N]).  Any pointer may be NULL.
 */
int fpc_macros(fpc_sim* s, double* rho, double* u, double* T);

/*
 * FP64 diagnostics of the current time level, reduced on the GPU with a fixed
 * (deterministic) order.  Synchronises the stream.  Host outputs (any may be NULL):
 *   nu_mean: mean wall Nusselt number on face `wall_face` (Sec. 6.1):
 *            dT/dn = -8/3 T_w + 3 T(1/2) - 1/3 T(3/2) along the inward normal,
 *            Nu = -(L / dT_ref) dT/dn, L = nodes along the face normal
 *            (pass wall_face = -1 to skip);
 *   ke:      1/2 sum rho |u|^2;   sumT: sum T;   umax: max |u|.
 * Returns FPC_ERR_UNSTABLE (outputs still written) if any macro is NaN/Inf or
 * umax exceeds 0.5.
 */
int fpc_diagnostics(fpc_sim* s, int wall_face, double* nu_mean, double* ke, double* sumT, double* umax);

/*
 * Local wall Nusselt numbers of the current time level on wall_face (the
 * stencil of fpc_diagnostics, Sec. 6.1, per wall node): nu[i] for wall node i
 * in the profile layout of fpc_params.wall_T_profile (the face's two
 * tangential axes, slower first); device pointer, M FP64 values.  Their mean
 * is fpc_diagnostics' nu_mean.  Asynchronous.  Errors as fpc_step_nusselt.
 */
int fpc_nusselt_local(fpc_sim* s, int wall_face, double* nu);

/*
 * The diagnostics of fpc_diagnostics without allocating, synchronising or
 * copying to the host: for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 * Writes out[0..4] = (mean wall Nusselt number on wall_face, or 0 for
 * wall_face = -1; KE; sum T; max |u|; number of nodes with a non-finite
 * macro), exactly the values fpc_diagnostics returns (same kernels, same
 * summation order), to `out` (device pointer, 5 FP64 values), asynchronously
 * on the simulation's stream.  The watchdog is left to the caller (out[4] != 0
 * or out[3] > 0.5).
 * The reduction partials live in a library-owned device array of
 * 1024 * 4 + 64 + 8 doubles (33 KiB) per GPU, held until the process ends;
 * the reductions use at most 1024 + 64 blocks, so every grid the library
 * accepts fits it (the call still returns FPC_ERR_SIZE if that bound were
 * ever exceeded).  Every call on one GPU shares that array: calls that overlap
 * on one GPU (other streams or host threads) race and must be serialised by
 * the caller.  Nothing in it needs clearing between calls.  Errors:
 * FPC_ERR_ARG (NULL sim or out, bad wall_face), FPC_ERR_STATE (periodic or
 * missing face), FPC_ERR_HIP (launch failure).
 */
int fpc_diagnostics_noalloc(fpc_sim* s, int wall_face, double* out);

/* Copy the current state (fpc_state_bytes() bytes, storage format) to / from
 * device memory.  fpc_load resets the step counter to `step`. */
int fpc_save(const fpc_sim* s, void* dst);
int fpc_load(fpc_sim* s, const void* src, long long step);

/* Current state as full FP64 populations (f = w rho0 + stored deviation in
 * FP32_DEV mode): (Qf + Qg) planes of N values, contiguous, no padding. */
int fpc_export_fp64(const fpc_sim* s, double* dst);
/* Replace the current state from full FP64 populations in the same layout. */
int fpc_import_fp64(fpc_sim* s, const double* src, long long step);

/* Device pointer of the buffer that holds the current state. */
int fpc_current_buffer(const fpc_sim* s, void** ptr);

/*
 * Adjoint seeds of the wall-Nusselt objective J = weight * <Nu>_face at one
 * time level (the stencil of Sec. 6.1 as in fpc_diagnostics):
 *   dJdT[x]  = dJ/dT(x): 3 s on the nodes next to the face, -s/3 on the second
 *              layer, 0 elsewhere, s = -(L / dT_ref) weight / M (M nodes on the
 *              face); device, N FP64 values [z][y][x], overwritten.  It is the
 *              dJdT argument of fpc_adjoint_step / fpc_adjoint_init.
 *   dJdTw[i] = dJ/dT_w(i) = -8/3 s, the direct dependence on the wall
 *              temperature of wall node i (profile layout of
 *              fpc_params.wall_T_profile); device, M FP64 values, overwritten;
 *              may be NULL.
 * Asynchronous.  Errors as fpc_step_nusselt.
 */
int fpc_nusselt_seed(fpc_sim* s, int wall_face, double weight, double* dJdT, double* dJdTw);

/*
 * Adjoint (reverse mode) of one time step S_n = Phi(S_{n-1}) = collide_n(
 * pull(S_{n-1})), for an objective J whose direct dependence on S_n is
 * through the time-n macros.  The adjoint is carried as mu: mu_n is the
 * adjoint of the pulled (pre-collision) populations entering the collision of
 * step n + 1, so that the adjoint of the stored state S_n is
 * lambda_n = pull^T mu_n.  Computes
 *   mu_out = mu_{n-1} = collide_n^T (pull^T mu_in + dJ/dS_n),  mu_in = mu_n,
 * where dJ/dS_n is formed in the kernel from
 *   dJdT[x]    weight of T_n(x)  (device, N FP64 values, or NULL), and
 *   ke_weight  weight of the kinetic energy 1/2 sum rho |u|^2 of time n,
 * and accumulates (+=) the gradient with respect to the per-node Dirichlet
 * wall temperature of face f into dJdtheta[f] (device, FP64, profile layout
 * of fpc_params.wall_T_profile; dJdtheta may be NULL, or hold NULL entries).
 * A reverse sweep starts from mu_N = 0 and ends with fpc_adjoint_init on
 * mu_0.  S_prev: S_{n-1} in storage format (fpc_state_bytes()).  mu_in,
 * mu_out: adjoint states in the same layout and element type as the state
 * (FP64 or FP32), distinct buffers; every element of mu_out that belongs to a
 * node is written (padding is not).  Each node reads mu_in along the reversed
 * links (the transpose of the pull, with the wall rules: -1 on Dirichlet
 * links) and writes only its own slots.  The method is not part of the paper:
 * this is the exact adjoint of the discrete update above, on every lattice
 * pair, model and thermal option.  On the D2Q9 / D3Q15 thermal lattices a
 * diagonal link crossing two or three Dirichlet faces (an edge or corner)
 * takes their mean temperature, so its gradient is split between them.
 */
int fpc_adjoint_step(fpc_sim* s, const void* S_prev, const void* mu_in, void* mu_out, const double* dJdT,
                     double ke_weight, double* const* dJdtheta);

/*
 * Adjoint of the initial collision (fpc_init): from mu0 (the adjoint of the
 * pulled populations of step 1, as left by the last fpc_adjoint_step of a
 * sweep) forms lambda_0 = pull^T mu0, adds the level-0 seed (dJdT, ke_weight
 * as in fpc_adjoint_step) and writes dJ/dT_init[x] (device, N FP64 values).
 */
int fpc_adjoint_init(fpc_sim* s, const double* T_init, const void* mu0, const double* dJdT, double ke_weight,
                     double* dJdT_init);

#ifdef __cplusplus
}
#endif

#endif /* FPCLBM_H */
