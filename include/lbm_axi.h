/*
 * lbm_axi -- axisymmetric MRT lattice Boltzmann for thermal flow in porous
 * media on AMD Instinct MI355X (gfx950).
 *
 * The library advances the model of Liu, He and Li (arXiv:1409.5929): the
 * r-weighted D2Q9 multiple-relaxation-time lattice for the flow (Sec. 3.1,
 * Eqs. 13-32) coupled to the D2Q5 lattice for the temperature (Sec. 3.2,
 * Eqs. 33-38), with the porous-medium body force of Eqs. (6)-(8) and the
 * relaxation times of Eq. (39).  One call of lbm_axi_step performs, per node
 * and time step, the fused update: macroscopic values (Eqs. 26-30, 38),
 * moment-space collision (Eqs. 16-25), back-transform and streaming (Eq. 22),
 * temperature collision and streaming (Eqs. 33-37).
 *
 * Conventions for every entry point:
 *   - Return value: LBM_AXI_OK (0) or a negative lbm_axi_error code; nothing
 *     aborts.  lbm_axi_last_error() gives a message for the calling thread.
 *   - Ownership: the caller owns every pointer it passes; inputs are copied
 *     before the call returns (device memory belongs to the handle).
 *   - Public 2-D arrays are C-ordered [nz][nr], r fastest, no padding.
 *   - A handle is not thread-safe; all its work runs on one HIP stream.
 *
 * Points the paper leaves open are settled as follows (the same readings the
 * test oracle takes; the paper's section is named for each):
 *   - Lattice: row j at radius r0 + j, column k at z = k, unit spacing
 *     (Sec. 4).  Wall nodes lie on the walls (rows 0, nr-1; columns 0, nz-1).
 *   - Walls: non-equilibrium extrapolation (Sec. 4): a wall node takes the
 *     equilibrium of (density of its fluid neighbour, zero velocity, wall
 *     temperature) plus the neighbour's non-equilibrium part, unscaled, and
 *     collides with those values.  The neighbour is the normal one, the
 *     diagonal one at corners.  Adiabatic walls copy the neighbour's
 *     temperature; isoflux walls (LBM_T_FLUX) add q'/k to it; at a corner a
 *     fixed-temperature radial wall wins.  Inlet and outlet columns
 *     (LBM_SIDE_FLOW, Sec. 4.1) are reconstructed the same way with their own
 *     velocity, density and temperature (see lbm_axi_side).
 *   - Axis (LBM_SIDE_AXIS at r_min, r0 must be 1/2): a mirror row at r = -1/2
 *     with f_i(-r) = -f_i*(r) for the r-weighted populations (i* reverses
 *     e_r) and g_i(-r) = g_i*(r).  It may be combined with axial walls or an
 *     inlet and outlet (pipes, closed cylinders).
 *   - Source moments: with src_printed = 0 the axisymmetric correction a_r of
 *     Eq. (25) enters the second-order moments of Eq. (24) without the 1/phi
 *     factor that the porous-medium force F carries; src_printed = 1 divides
 *     all of F~ by phi exactly as Eq. (24) is printed (equal when phi = 1).
 *   - Start: f = f^eq - S~/2 at rho = 1 (the change of variables before
 *     Eq. 15), g = g^eq (Eq. 35).
 *   - Buoyancy (Eq. 7) along +z with g*beta*dT = (Ma c_s)^2 / L when Ra > 0.
 *   - Variable porosity: K(x) from Eq. (8) with the particle diameter fixed by
 *     K(phi) = Da L^2 at the reference porosity p.phi; F_phi < 0 selects the
 *     Ergun coefficient of Eq. (8) from the local porosity.
 */
#ifndef LBM_AXI_H
#define LBM_AXI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_axi lbm_axi;

enum lbm_axi_error {
  LBM_AXI_OK = 0,
  LBM_AXI_EINVAL = -1,       /* invalid argument or parameter */
  LBM_AXI_ENOMEM = -2,       /* device or host allocation failed */
  LBM_AXI_EDEVICE = -3,      /* a HIP call failed (message names it) */
  LBM_AXI_EUNSUPPORTED = -4  /* a parameter value the model does not define */
};

/*
 * LBM_SIDE_FLOW (side_z only) makes column 0 a velocity inlet and column
 * nz-1 an outlet (Sec. 4.1), both reconstructed like walls: the inlet node
 * takes u = (u_r, u_z) = (0, u_in), T = T_zmin when therm_z is fixed (else its
 * neighbour's T) and its neighbour's density; the outlet node takes its
 * neighbour's u and T (zero axial gradient) and rho = rho_0 = 1, which fixes
 * the pressure level the paper leaves open.  Radial walls win at corners.
 */
enum lbm_axi_side {
  LBM_SIDE_WALL = 0,     /* no-slip wall, nodes on the wall */
  LBM_SIDE_AXIS = 1,     /* axis of symmetry; r_min only */
  LBM_SIDE_PERIODIC = 2, /* periodic; along r only for tests (both r sides) */
  LBM_SIDE_FLOW = 3      /* z only: inlet at z_min, outlet at z_max */
};

/*
 * Thermal wall types.  LBM_T_FLUX (radial walls only) is the isoflux wall of
 * Sec. 4.4: the nodes of the wall with flux_zlo <= z <= flux_zhi carry the
 * heat flux q' = -k dT/dn into the fluid (n the outward normal of the fluid,
 * so q' = -k dT/dr on an r_min wall) and the rest of the wall is adiabatic.
 * A heated wall node takes T_b = T_B + q'/k, the one-sided difference to its
 * fluid neighbour B one spacing away, and is then treated like any wall node;
 * at a corner a fixed-temperature wall wins.
 */
enum lbm_axi_thermal { LBM_T_FIXED = 0, LBM_T_ADIABATIC = 1, LBM_T_FLUX = 2 };

/* Storage of the populations.  Arithmetic is FP32 in every case. */
enum lbm_axi_storage {
  LBM_STORE_FP32 = 0,
  LBM_STORE_FP16 = 1, /* shifted: deviation from the rest state, scaled by 2^storage_shift */
  LBM_STORE_BF16 = 2
};

/* Per-instance run state reported by lbm_axi_residual. */
enum lbm_axi_run_state {
  LBM_RUNNING = 0,
  LBM_CONVERGED = 1, /* residual <= tol, or exactly 0 */
  LBM_DIVERGED = 2,  /* residual NaN or infinite */
  LBM_STALLED = 3    /* max_steps reached */
};

/*
 * Problem statement of one instance.  Lattice units: dt = dr = dz = 1.
 * lbm_axi_default_params fills the paper's defaults (Sec. 4): J = lambda = 1,
 * Ma = 0.1, s_e = s_eps = 1.1, s_q = 1.2, s_j = 1, sigma = 1.
 */
typedef struct lbm_axi_params {
  int32_t nr, nz;              /* grid: rows along r, columns along z (>= 3 each with walls) */
  int32_t side_rmin, side_rmax, side_z;      /* lbm_axi_side */
  int32_t therm_rmin, therm_rmax, therm_z;   /* lbm_axi_thermal */
  int32_t storage;             /* lbm_axi_storage */
  int32_t storage_shift;       /* power-of-two scale of shifted storage (FP16: default 10) */
  int32_t check_interval;      /* residual / Nusselt check every N steps (>= 2; 0 = never) */
  int32_t src_printed;         /* 1: Eq. (24) exactly as printed (see above) */
  double r0;                   /* radius of row 0 (> 0; 1/2 with an axis) */
  double L;                    /* characteristic length of Eq. (9) */
  double phi;                  /* porosity; reference porosity when a field is given */
  double Da;                   /* Darcy number K / L^2 (Eq. 9) */
  double F_phi;                /* Forchheimer coefficient of Eq. (6); < 0: Ergun, Eq. (8) */
  double Ra, Pr, J, lambda;    /* Eq. (9) groups; Ra > 0 turns buoyancy on */
  double sigma;                /* heat-capacity ratio: only 1 is defined (Eq. 4) */
  double Ma;                   /* Mach number of Eq. (39) */
  double tau_nu;               /* > 0 overrides tau_nu of Eq. (39) */
  double accel_r, accel_z;     /* external acceleration a of Eq. (7) */
  double s_e, s_eps, s_q, s_j; /* relaxation rates of Eq. (23); s_nu = 1 / tau_nu */
  double T_rmin, T_rmax, T_zmin, T_zmax; /* temperatures of fixed-temperature walls */
  double T_ref;                /* reference temperature T_0 of Eq. (7) */
  double T_init;               /* initial temperature where no field is given */
  double delta_T;              /* temperature difference of Ra and Nu; 0: T_rmin - T_rmax */
  double tol;                  /* convergence threshold on the residual (0: only an exact 0) */
  int64_t max_steps;           /* stall after this many steps (0: never) */
  double flux_rmin, flux_rmax; /* q'/k of LBM_T_FLUX walls (temperature per lattice unit) */
  double flux_zlo, flux_zhi;   /* heated window of LBM_T_FLUX walls in z (default: all) */
  double u_in;                 /* inlet axial velocity with side_z = LBM_SIDE_FLOW */
  double tail_tol;             /* > 0: convergence also needs the extrapolated tail (below) <= tail_tol */
} lbm_axi_params;

/* Fill *p with the paper's default rates and ratios; grid and physics zero. */
void lbm_axi_default_params(lbm_axi_params* p);

/*
 * Create n_inst independent instances (p points to n_inst parameter blocks)
 * and set them to the start state.  phi_field: NULL, or n_inst host pointers,
 * each NULL (uniform p.phi) or [nz][nr] floats with 0 < phi < 1.  init_uzurT:
 * NULL, or n_inst host pointers, each NULL (rest, T_init) or [3][nz][nr]
 * floats (u_z, u_r, T).  hip_stream: the hipStream_t to run on (NULL: the
 * library creates one).  On failure *out is NULL and device memory is freed.
 * Every instance must use the same check_interval.
 */
int lbm_axi_create(const lbm_axi_params* p, int32_t n_inst, const float* const* phi_field,
                   const float* const* init_uzurT, void* hip_stream, lbm_axi** out);

/*
 * Advance every running instance by nsteps time steps (asynchronous on the
 * handle's stream).  At every multiple of check_interval (from the second
 * one on, counting step 0) the residual and the wall Nusselt numbers are
 * computed on the device and the run state updated; instances that stop are
 * skipped from then on.
 */
int lbm_axi_step(lbm_axi* h, int32_t nsteps);

/*
 * Macroscopic fields of instance inst at its current time (pre-collision):
 * u_z, u_r, p = rho c_s^2 / phi and T (Eqs. 26-28, 38 and the text after
 * Eq. 30), and the node classes (bit 0 r_min wall, 1 r_max wall, 2 z_min
 * wall, 3 z_max wall, 4 row next to the axis).  Each pointer may be NULL.
 * Wall nodes report u = 0, their wall temperature and the density of the
 * neighbour they are built from.  dst_is_device: 1 if the pointers are device
 * memory (written on the handle's stream, not waited for), 0 for host memory
 * (the call waits).
 */
int lbm_axi_macros(lbm_axi* h, int32_t inst, float* uz, float* ur, float* p, float* T,
                   uint8_t* mask, int32_t dst_is_device);

/*
 * Density deviation rho - 1 of instance inst at its current time (Eq. 26;
 * the rest density is 1), into drho ([nz][nr] floats).  The library keeps
 * populations as deviations from the rest state, so this value carries FP32's
 * relative precision even where rho is within 1e-6 of 1, which the total
 * p = rho c_s^2 / phi of lbm_axi_macros cannot resolve.  Wall nodes report the
 * density they are built from (lbm_axi_macros).  dst_is_device as in
 * lbm_axi_macros.  LBM_AXI_EINVAL if drho is NULL.
 */
int lbm_axi_density_deviation(lbm_axi* h, int32_t inst, float* drho, int32_t dst_is_device);

/*
 * Stokes stream function of instance inst at its current time (the paper
 * reports its largest magnitude in Table 3 without defining it):
 * u_z = (1/r) dpsi/dr, u_r = -(1/r) dpsi/dz, psi = 0 on the r_min wall, i.e.
 * psi(r_j, z_k) = integral from r0 to r_j of r u_z dr by the trapezoid rule
 * over the rows (FP64 sums of the FP32 velocity field); with an axis at r_min
 * psi = 0 on the axis and the integral starts at r = 0 (row 0 holds
 * r0 (r0 u_z) / 2, the trapezoid over [0, r0]).  In lattice units; divide
 * by alpha_e L, alpha_e = c_sT^2 tau_T the effective thermal diffusivity
 * (text after Eq. 38), for the scale of Table 3 (the paper does not state
 * it; this one matches its values at Da = 1e-4 and 1e-2, nu L does not).
 * psi: NULL or [nz][nr] floats, device memory if dst_is_device (written on
 * the handle's stream) else host memory.  psi_absmax: NULL or one host double, max |psi|.  The
 * call allocates temporary device memory and waits for the stream.
 */
int lbm_axi_stream_function(lbm_axi* h, int32_t inst, float* psi, double* psi_absmax,
                            int32_t dst_is_device);

/*
 * lbm_axi_stream_function for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result without any allocation.  psi: NULL or device
 * memory for [nz][nr] floats; psi_absmax: NULL or device memory for one
 * double (max |psi|).  Both are written on the handle's stream and not waited
 * for.  Its scratch (the u_z field and the per-column maxima) is a static
 * array of the library on each device, held until the process ends, of at
 * most 2^23 nodes and 2^16 columns: a larger instance gets LBM_AXI_EINVAL.
 * All handles on one device share that array and each call leaves its
 * contents behind, so calls that overlap on one device (handles on different
 * streams, threads) race; calls ordered on one stream do not.  The call reads
 * the instance's run state and time level from the device (a small copy to
 * the host, as lbm_axi_info).
 */
int lbm_axi_stream_function_static(lbm_axi* h, int32_t inst, float* psi, double* psi_absmax);

/*
 * Local Nusselt number along the wall of a pipe (axis at r_min, wall at
 * r_max), Sec. 4.1: at each column k, Nu = D (dT/dr)_w / (T_w - T_b) (Eq. 40)
 * with D = 2 r_w and the second-order one-sided wall gradient.  T_b is the
 * bulk temperature: with area = 0 the mixing-cup value
 * int r u_z T dr / int r u_z dr (the bulk temperature of the textbook pipe
 * Nusselt numbers the paper's Table 1 reproduces), with area = 1 the area
 * mean int r T dr / int r dr as Eq. (41) is printed; the integrals run from
 * the axis to the wall by the trapezoid rule over the rows plus the point
 * r = 0.  FP64 sums of the FP32 fields at the instance's current time.  nu
 * and T_b are host arrays of nz doubles (each may be NULL).  A column that
 * carries no net axial flux (a closed cylinder) has no mixing-cup T_b: its
 * entries then divide by a vanishing flux and carry no meaning (use area = 1).  Allocates temporary device memory and waits
 * for the stream.  LBM_AXI_EINVAL unless the instance is a pipe.
 */
int lbm_axi_pipe_nusselt(lbm_axi* h, int32_t inst, int32_t area, double* nu, double* T_b);

/*
 * Latest check of every instance (waits for the stream).  Each pointer may be
 * NULL; arrays have n_inst entries.  The paper defines no convergence
 * criterion; at step n (a multiple N of check_interval) res = max(R_u, R_T)
 * with R_u = rms over the fluid nodes of |u^n - u^{n-N}| / N divided by the
 * characteristic velocity Ma c_s (text before Eq. 39) and R_T the same for T
 * divided by dT (FP64 sums): the mean change per step over the interval, so
 * that rounding flicker of FP32 storage does not set a floor.  nu_i, nu_o =
 * Eq. (42) at step n on the r_min and r_max walls (second-order one-sided
 * dT/dr, trapezoid rule, H = nz - 1).  status = lbm_axi_run_state.  Before
 * the first check res = +inf.  On an LBM_T_FLUX wall nu_i (nu_o) is instead
 * the heater mean of Eqs. (43)-(44): Nu(z) = (q'/k) L / (T_h - T_ref) at each
 * heated wall node (T_h its wall temperature; the paper takes T_0 = T_o, the
 * cold-wall temperature), averaged over the heated nodes (NaN if none).
 * Convergence: res <= tol.  A residual measures the rate of change, and an
 * instance that relaxes slowly (time constant tau steps) stops at res = tol
 * still about tau * tol away from its steady state.  With tail_tol > 0 it
 * must also bring the changes still to come, extrapolated geometrically from
 * its last checks, to at most tail_tol, each of: R_u N rho / (1 - rho) and
 * R_T N rho / (1 - rho) (rho the ratio of the part's last two values,
 * infinite while rho >= 1; units of res times steps, i.e. a distance to the
 * steady state relative to U and dT), and for Nu_i and Nu_o the change over
 * the last interval times rho / (1 - rho), relative to Nu (rho the ratio of
 * the last two interval changes; a change below 1e-7 Nu counts as none).
 */
int lbm_axi_residual(lbm_axi* h, double* res, double* nu_i, double* nu_o, int32_t* status);

/*
 * Details of instance inst (waits for the stream): out[0] = its own time
 * level (the steps it has taken: the handle's level while it runs, the level
 * at which it stopped once it has stopped, less the handle steps it sat out
 * before a restart by lbm_axi_set_storage), out[1] = handle level of its
 * latest check, out[2] = run state, out[3] = bytes of device memory the
 * handle holds.  out has 4 entries.
 */
int lbm_axi_info(lbm_axi* h, int32_t inst, int64_t* out);

/*
 * Constants the library derives from a problem statement (FP64, on the host;
 * needs no device and no handle): out[0] = tau_nu and out[1] = tau_T of
 * Eq. (39) (tau_nu as given when p->tau_nu > 0), out[2] = nu_e (Eq. 31),
 * out[3] = nu = nu_e / J and out[4] = K = Da L^2 (Eq. 9), out[5] = g beta =
 * (Ma c_s)^2 / (L dT) (0 without buoyancy), out[6] = alpha_e = c_sT^2 tau_T
 * (text after Eq. 38).  out has 7 entries.  LBM_AXI_EINVAL on NULL.
 */
int lbm_axi_derived(const lbm_axi_params* p, double* out);

/*
 * Streaming ceiling of the step's memory access pattern, measured on the
 * handle's own arrays and launch shapes (waits for the stream): probe kernels
 * that make exactly the step kernel's loads and stores for each parity of the
 * in-place (AA) layout, with no arithmetic (every value is stored back where
 * it was read, so the state is unchanged), and a plain in-place read+write
 * stream over the population arrays.  Each is launched reps times after one
 * untimed launch and timed with HIP events on the handle's stream.
 * out[0] = even-step pattern, out[1] = odd-step pattern, out[2] = plain
 * stream, in GB/s (bytes read plus written per second; the patterns count the
 * step's algorithmic bytes: per fluid node of the running instances, 13
 * populations of the storage type and the FP32 g_0 read and written, and the
 * porosity read where it is a field), out[3] = those algorithmic bytes of one
 * step launch.  out has 4 entries; 1 <= reps <= 100000.
 */
int lbm_axi_pattern_bandwidth(lbm_axi* h, int32_t reps, double* out);

/*
 * Lane-width probe (no part of the method): an in-place read+write stream
 * over every instance's population array (bits XORed with 0, so the state
 * is unchanged) with lanes of 2, 4, 8 and 16 bytes, reps timed passes each
 * after an untimed one.  out[0..3] = GB/s (bytes read plus written per
 * second) for the four widths.  The same bytes at narrower lanes take more
 * memory instructions; the 16-bit storage layout pairs slots in 4-byte words
 * for this reason.  Waits for the stream; 1 <= reps <= 100000.
 */
int lbm_axi_lane_bandwidth(lbm_axi* h, int32_t reps, double* out);

/*
 * Kernel timing: with on = 1 every later step-kernel launch is bracketed by
 * HIP events on the handle's stream; lbm_axi_kernel_time returns the summed
 * milliseconds and the number of launches since timing was switched on
 * (waits for the stream).  on = 0 stops timing.
 */
int lbm_axi_set_timing(lbm_axi* h, int32_t on);
int lbm_axi_kernel_time(lbm_axi* h, double* total_ms, int64_t* launches);

/*
 * Launch shape of the step kernel: blocks of 64 lanes along r by 4 waves,
 * each thread updating kz nodes along z (1 <= kz <= 64), and at most
 * blocks_per_cu blocks resident per compute unit (0: no cap; 1..64).  This
 * call sets the same kz for both parities of the AA step.  By default each
 * parity has its own: the largest of 1 (FP32 even steps), 2 (FP32 odd steps)
 * or 8 (16-bit storage), halving down to 1, that gives the launch at least
 * 512 blocks (short strips for small, latency-bound grids); a storage
 * conversion re-applies the default unless this call or lbm_axi_autotune
 * chose the shape.
 * Waits for the stream and rebuilds the tile lists; results do not depend
 * on it.
 */
int lbm_axi_set_tiles(lbm_axi* h, int32_t kz, int32_t blocks_per_cu);

/*
 * Which lanes compute the radial no-slip wall nodes beside fluid rows
 * (non-equilibrium extrapolation, Sec. 4).  With wall lanes (mode 1) each
 * such wall node's own lane, idle otherwise, loads its owner's populations
 * with the owner's wave and writes the wall populations that stream into
 * fluid nodes; without (mode 0) the owner writes them after its own update,
 * which costs a wave about twice an interior wave but keeps the kernel's
 * register count lower.  mode -1 restores the default, chosen once from the
 * instances: wall lanes when more than 5 % of the step's waves (64-column
 * groups, weighted by nz) hold a wall lane, as for batches of grids a few
 * hundred columns wide, not for one 8192^2 grid.  The two variants give the
 * same results up to FP32 rounding of the wall populations (and different
 * random bits for their 16-bit stores), so a run is bit-reproducible only
 * within one setting.  *on (nullable) receives the setting in force (0/1).
 * Waits for the stream and drops a captured step graph.
 */
int lbm_axi_set_wall_lanes(lbm_axi* h, int32_t mode, int32_t* on);

/*
 * Change the storage type of every instance's populations (LBM_STORE_*),
 * keeping the state: each slot keeps its value, converted to the new type
 * (rounded to nearest), with temperature slots moved to the new type's shift.
 * storage_shift means what it means in the parameter struct (0: the type's
 * default; 0..24).  The intended use is a precision handoff: iterate in
 * 16-bit storage while the solution still changes by more than the storage
 * noise, then finish in FP32.
 * Waits for the stream; allocates the new arrays before freeing the old ones,
 * so on LBM_AXI_ENOMEM the handle is unchanged.  Step count, the last check
 * and the check buffers carry over.  Converged instances are set running
 * again from the state at which they stopped: one whose stopping level and
 * the handle's current level differ in parity first takes one step on its
 * own, so that its in-place (AA) layout matches the handle's; the handle steps
 * it sat out do not count as its steps (lbm_axi_info), and its first check
 * after the restart records the Nusselt numbers only (residual +inf), since
 * a residual needs a full check interval of its own steps.  Stalled and
 * diverged instances stay stopped.
 */
int lbm_axi_set_storage(lbm_axi* h, int32_t storage, int32_t storage_shift);

/*
 * Step graphs: lbm_axi_step sends every run of `steps` consecutive plain
 * steps (starting at an even time level, no check step inside) through one
 * captured HIP graph, replayed on the handle's stream; check steps and the
 * rest are launched one by one.  Results are identical either way.  steps is
 * even, 0..4096; 0 disables graphs; default 32.  Launch timing
 * (lbm_axi_set_timing) bypasses the graphs.  Waits for the stream.
 */
int lbm_axi_set_graph(lbm_axi* h, int32_t steps);

/*
 * Drops instances that are no longer running (converged, diverged, stalled)
 * from the step launch, so that a batch whose instances finish at different
 * times stops paying for the finished ones.  Reads the run states (waits for
 * the stream).  *n_running (may be NULL) receives the number still running.
 */
int lbm_axi_compact(lbm_axi* h, int32_t* n_running);

/*
 * Autotuner of the step launch: runs trial_steps real steps (they advance
 * the solution) with each candidate launch shape (nodes per thread along z
 * in {1, 2, 4, 8, 16} x resident-block cap in {none, 2, 4} per compute unit),
 * timing every step launch with HIP events, and keeps the fastest.  The
 * chosen shape and its mean step-launch time (ms) are returned through the
 * pointers (each may be NULL).  15 x trial_steps steps are taken in all.
 */
int lbm_axi_autotune(lbm_axi* h, int32_t trial_steps, int32_t* kz_out, int32_t* bpc_out,
                     double* ms_out);

/* Wait for the handle's stream. */
int lbm_axi_sync(lbm_axi* h);

/* Free everything the handle holds.  NULL is allowed. */
void lbm_axi_destroy(lbm_axi* h);

/* Message of the last failed call on this thread ("" if none). */
const char* lbm_axi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_AXI_H */
