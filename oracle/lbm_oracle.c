/*
 * FP64 CPU oracle of the axisymmetric MRT lattice Boltzmann model for thermal
 * flow in porous media of Liu, He and Li (arXiv:1409.5929).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference for the GPU
 * library.  Only the test suite, the package smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or constant
 * with the GPU library, and the GPU library never calls it.
 *
 * It is written to be checked against the paper by eye, not to be fast:
 *   - populations are the paper's r-weighted f_i (Eq. 17, Eq. 26) and the
 *     plain temperature populations g_i (Eq. 38), stored node by node;
 *   - every moment transform is a dense 9x9 product with the printed matrix M
 *     (Eq. 18) and its inverse, obtained here by Gauss-Jordan elimination;
 *   - one time step = macroscopic quantities (Eqs. 26-30, 38), collision in
 *     moment space (Eqs. 19-25, 21), back-transform (Eq. 22), temperature
 *     collision (Eqs. 33-37), then streaming of both lattices (Eq. 22, Eq. 33)
 *     from a post-collision copy into a fresh array (two-array scheme).
 *
 * Readings of points the paper leaves open (the GPU library takes the same
 * readings, written independently):
 *   R1 Lattice and walls.  Row j sits at radius r_j = r0 + j, column k at
 *      z = k, with unit spacing (Sec. 4 preamble: all spacings are 1).  Wall
 *      nodes lie on the walls: rows 0 and nr-1, columns 0 and nz-1.
 *   R2 Walls use non-equilibrium extrapolation (Sec. 4 preamble, the paper's
 *      ref. [47]): a wall node b takes the equilibrium of the wall state
 *      (density of its fluid neighbour B, zero velocity, wall temperature) plus
 *      the non-equilibrium part of B's populations, unscaled, and then
 *      collides like any node with those imposed macroscopic values.  B is the
 *      normal neighbour; a corner uses its diagonal neighbour.  Adiabatic walls
 *      copy B's temperature.  At a corner a fixed-temperature radial wall wins
 *      over an axial wall.
 *   R3 Axis of symmetry (pipe).  The paper is silent on it.  Rows are
 *      cell-centred (r0 = 1/2) and a ghost row at r = -1/2 mirrors row 0.
 *      Since f = r * fhat with fhat symmetric about the axis, the mirrored
 *      r-weighted populations change sign: f_i(-r) = -f_i*(r), i* = the
 *      direction with e_r reversed.  The temperature populations are mirrored
 *      without sign change.
 *   R4 Eq. (28) is applied literally, also when l_r0 != l_z0.
 *   R5 The axial buoyancy is +z, G_z = g*beta*(T - T_ref) (Eq. 7), with
 *      g*beta*dT = U^2/L and U = Ma*c_s (text before Eq. 39) when Ra > 0, and
 *      no buoyancy when Ra = 0.
 *   R6 Variable porosity: K(x) follows Eq. (8) with the particle diameter
 *      fixed so that K(phi_ref) = Da*L^2; F_phi(x) = 1.75/sqrt(150 phi(x)^3)
 *      when the given F_phi is negative (Ergun, Eq. 8).
 *   R7 Source moments.  As printed, Eq. (24) divides every product of u with
 *      F~ = F + a_r (Eq. 25) in the second-order moments by phi.  The part
 *      a_r = c_s^2 [1 - 2(tau-1/2) u_r / r] / r is the axisymmetric
 *      correction, not a porous-medium force: it balances the radial flux of
 *      the r-weighted equilibrium, which carries no phi.  Taken as printed,
 *      the model does not recover Eq. (11) when phi != 1 (Hagen-Poiseuille
 *      pipe flow at phi = 0.6 comes out 1.5 times too fast), although
 *      Appendix A states that it does.  The default (src_printed = 0) divides
 *      only F by phi and keeps a_r unscaled: at phi = 1 both forms coincide,
 *      and with it the porous pipe converges to the Brinkman solution at
 *      second order.  src_printed = 1 evaluates Eq. (24) exactly as printed.
 *   R8 Initial state (not given in the paper).  The implicit populations
 *      start at equilibrium, f~ = f^eq(rho = 1, u0), and the explicit ones
 *      follow from the change of variables that leads to Eq. (15),
 *      f = f~ - (dt/2) S~, i.e. f = M^{-1} (m^eq - S/2).  Then Eqs. (26)-(28)
 *      return u0 itself (exactly when F_phi = 0).  g = g^eq(T0, u0).
 *   R9 Isoflux walls (Sec. 4.4).  A radial wall of type THERM_FLUX carries the
 *      heat flux q' = -k dT/dn (n pointing out of the fluid, so dT/dr at r_min)
 *      on its nodes with flux_zlo <= z <= flux_zhi and is adiabatic elsewhere.
 *      The given flux is q'/k, a temperature gradient.  A heated wall node
 *      takes T_b = T_B + (q'/k) * 1, the one-sided difference to its fluid
 *      neighbour B one spacing away (the adiabatic copy T_b = T_B is the case
 *      q' = 0), and is then treated as in R2.  At a corner any
 *      fixed-temperature wall wins over the flux.
 *   R10 Heater Nusselt numbers (Eqs. 43-44).  Nu(z) = (q'/k) L / (T_h - T_0)
 *      at each heated node, T_h its wall temperature and T_0 = T_ref (the
 *      paper takes T_0 = T_o, the cold wall); the heater mean is the plain
 *      average over the heated nodes, each standing for a unit length of
 *      wall (midpoint rule of Eq. 43).
 *   R12 Inlet and outlet (Sec. 4.1).  With side_z = SIDE_FLOW, column 0 is a
 *      velocity inlet and column nz-1 an outlet, both reconstructed as in R2
 *      with their own macroscopic state: the inlet takes u = (0, u_in),
 *      T = T_zmin (when therm_z is fixed; else B's T) and B's density; the
 *      outlet takes B's velocity and temperature (zero axial gradient, as the
 *      paper states) and rho = rho_0 = 1 (the paper leaves the pressure level
 *      open; fixing it at the outlet is the usual choice).  Radial walls win
 *      at the corners (no slip, and their temperature when fixed).
 *   R13 Pipe Nusselt number (Eqs. 40-41) at each column: D (dT/dr)_w /
 *      (T_w - T_b) with D = 2 r_w and the second-order one-sided gradient of
 *      Eq. (42) on the r_max wall.  The paper calls T_b the bulk temperature,
 *      and its clear-pipe value is the textbook 3.657, which holds for the
 *      mixing-cup temperature T_b = int r u_z T dr / int r u_z dr.  The
 *      printed Eq. (41) lacks the u_z weight: with it, the fully developed
 *      clear pipe gives about 5.6 instead.  So T_b is the mixing-cup value by
 *      default; the printed area mean int r T dr / int r dr is available as
 *      the other weighting.  Both integrals run from the axis to the wall by
 *      the trapezoid rule over the rows plus the point r = 0 (where the
 *      integrand vanishes).
 *   R11 Stream function (Table 3; not defined in the paper).  The Stokes
 *      stream function of the axisymmetric flow, u_z = (1/r) dpsi/dr and
 *      u_r = -(1/r) dpsi/dz, zero on the r_min wall (or on the axis r = 0):
 *      psi(r, z) = integral from r_min (or 0) to r of r' u_z(r', z) dr'.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- lattice constants --------------------------------------------------- */
#define DT 1.0            /* time step (Sec. 4 preamble) */
#define CS2 (1.0 / 3.0)   /* c_s^2 for D2Q9 with c = 1 (text after Eq. 25) */
#define CST2 (1.0 / 5.0)  /* c_sT^2 for D2Q5 with omega_0 = 3/5 (after Eq. 36) */

/* Eq. (14): D2Q9 velocities in (r, z) order. */
static const int EX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EZ9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Eq. (34): D2Q5 velocities; Eq. (36) weights with omega_0 = 3/5. */
static const int EX5[5] = {0, 1, 0, -1, 0};
static const int EZ5[5] = {0, 0, 1, 0, -1};
static const double W5[5] = {0.6, 0.1, 0.1, 0.1, 0.1};

/* Eq. (18): the transformation matrix M. */
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},         {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},     {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},      {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},      {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

enum { SIDE_WALL = 0, SIDE_AXIS = 1, SIDE_PERIODIC = 2, SIDE_FLOW = 3 };
enum { THERM_FIXED = 0, THERM_ADIABATIC = 1, THERM_FLUX = 2 };
enum { MASK_RMIN = 1, MASK_RMAX = 2, MASK_ZMIN = 4, MASK_ZMAX = 8, MASK_AXISROW = 16 };

typedef struct {
  int32_t nr, nz;
  int32_t side_rmin, side_rmax, side_z;
  int32_t therm_rmin, therm_rmax, therm_z;
  double r0;       /* radius of row 0 */
  double L;        /* characteristic length */
  double phi;      /* porosity (reference porosity when a field is given) */
  double Da;       /* Darcy number K/L^2 (Eq. 9) */
  double F_phi;    /* Forchheimer coefficient; negative = Ergun (Eq. 8) */
  double Ra, Pr, J, lambda, Ma;
  double tau_nu;   /* > 0 overrides Eq. (39) */
  double accel_r, accel_z; /* external acceleration a of Eq. (7) */
  double s_e, s_eps, s_q, s_j; /* Eq. (23) rates; s_nu = 1/tau_nu */
  double s_nu;     /* > 0 overrides 1/tau_nu for s_7, s_8 (pin tests only) */
  int32_t src_printed; /* 1: Eq. (24) exactly as printed; 0: reading R7 */
  double T_rmin, T_rmax, T_zmin, T_zmax;
  double T_ref;    /* T_0 of Eq. (7) */
  double T_init;   /* initial temperature where no field is given */
  double delta_T;  /* characteristic temperature difference; 0 = T_rmin - T_rmax */
  double flux_rmin, flux_rmax; /* q'/k of THERM_FLUX radial walls (R9) */
  double flux_zlo, flux_zhi;   /* heated window of a flux wall, z = k */
  double u_in;                 /* inlet axial velocity of SIDE_FLOW (R12) */
} orc_params;

typedef struct {
  orc_params p;
  double tau_nu, tau_T, nu_e, nu, K_ref, gbeta;
  double lam[9];
  double Minv[9][9];
  int nr, nz, n;
  double* r;          /* [nr] */
  double *phi, *K, *Fphi; /* [n] */
  double *f, *g;      /* [n][9], [n][5] pre-collision populations at time t */
  double *fp, *gp;    /* post-collision scratch */
  double *fn, *gn;    /* streaming destination */
  double *rho, *ur, *uz, *T; /* macroscopic values at time t */
  double *pur, *puz, *pT;    /* macroscopic values at the snapshot time */
  long t_snap;
  int have_prev;
  uint8_t* mask;
  long t;
} orc_state;

/* ---- M^{-1} by Gauss-Jordan elimination with partial pivoting ------------ */
static int invert9(const double A[9][9], double X[9][9]) {
  double a[9][18];
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 18; ++j) a[i][j] = (j < 9) ? A[i][j] : (j - 9 == i ? 1.0 : 0.0);
  for (int c = 0; c < 9; ++c) {
    int piv = c;
    for (int i = c + 1; i < 9; ++i)
      if (fabs(a[i][c]) > fabs(a[piv][c])) piv = i;
    if (fabs(a[piv][c]) < 1e-300) return -1;
    if (piv != c)
      for (int j = 0; j < 18; ++j) {
        double tmp = a[c][j];
        a[c][j] = a[piv][j];
        a[piv][j] = tmp;
      }
    double d = a[c][c];
    for (int j = 0; j < 18; ++j) a[c][j] /= d;
    for (int i = 0; i < 9; ++i) {
      if (i == c) continue;
      double m = a[i][c];
      if (m != 0.0)
        for (int j = 0; j < 18; ++j) a[i][j] -= m * a[c][j];
    }
  }
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) X[i][j] = a[i][j + 9];
  return 0;
}

static void matvec9(const double A[9][9], const double* x, double* y) {
  for (int i = 0; i < 9; ++i) {
    double s = 0.0;
    for (int j = 0; j < 9; ++j) s += A[i][j] * x[j];
    y[i] = s;
  }
}

/* ---- per-node physics ----------------------------------------------------- */

/* Eq. (7): buoyancy plus external acceleration. */
static void body_accel(const orc_state* s, double T, double* Gr, double* Gz) {
  *Gr = s->p.accel_r;
  *Gz = s->gbeta * (T - s->p.T_ref) + s->p.accel_z;
}

/* Eqs. (19)-(20) multiplied by r as in Eq. (19). */
static void eq_moments(double r, double rho, double ur, double uz, double phi, double* meq) {
  double u2 = ur * ur + uz * uz;
  meq[0] = r * rho;
  meq[1] = r * (-2.0 * rho + 3.0 * rho * u2 / phi);
  meq[2] = r * (rho - 3.0 * rho * u2 / phi);
  meq[3] = r * rho * ur;
  meq[4] = r * (-rho * ur);
  meq[5] = r * rho * uz;
  meq[6] = r * (-rho * uz);
  meq[7] = r * rho * (ur * ur - uz * uz) / phi;
  meq[8] = r * rho * ur * uz / phi;
}

/* Eq. (24) with F~ = (F_r + a_r, F_z) of Eq. (25); reading R7 unless printed. */
static void source_moments(int printed, double r, double rho, double ur, double uz, double phi,
                           double Fr, double Fz, double ar, double* S) {
  double Ftr = Fr + ar, Ftz = Fz;
  S[0] = 0.0;
  S[3] = r * rho * Ftr;
  S[4] = r * rho * (-Ftr);
  S[5] = r * rho * Ftz;
  S[6] = r * rho * (-Ftz);
  if (printed) {
    double uF = ur * Ftr + uz * Ftz;
    S[1] = r * rho * 6.0 * uF / phi;
    S[2] = r * rho * (-6.0 * uF / phi);
    S[7] = r * rho * 2.0 * (ur * Ftr - uz * Ftz) / phi;
    S[8] = r * rho * (ur * Ftz + uz * Ftr) / phi;
  } else {
    double uF = ur * Fr + uz * Fz;
    S[1] = r * rho * 6.0 * (uF / phi + ur * ar);
    S[2] = r * rho * (-6.0 * (uF / phi + ur * ar));
    S[7] = r * rho * 2.0 * ((ur * Fr - uz * Fz) / phi + ur * ar);
    S[8] = r * rho * ((ur * Fz + uz * Fr) / phi + uz * ar);
  }
}

/* Eq. (6), the total force, and a_r of Eq. (25), its axisymmetric correction. */
static void total_force(const orc_state* s, double r, double phi, double K, double Fphi,
                        double ur, double uz, double T, double* Fr, double* Fz, double* ar) {
  double Gr, Gz;
  body_accel(s, T, &Gr, &Gz);
  double umag = sqrt(ur * ur + uz * uz);
  *Fr = -phi * s->nu / K * ur - phi * Fphi / sqrt(K) * umag * ur + phi * Gr;
  *Fz = -phi * s->nu / K * uz - phi * Fphi / sqrt(K) * umag * uz + phi * Gz;
  *ar = CS2 * (1.0 - 2.0 * (s->tau_nu - 0.5) * DT * ur / r) / r;
}

/* Eqs. (26)-(30) and (38): density, velocity and temperature of one node. */
static void node_macros(const orc_state* s, double r, double phi, double K, double Fphi,
                        const double* f, const double* g, double* rho, double* ur,
                        double* uz, double* T) {
  double sum = 0.0, jr = 0.0, jz = 0.0, tsum = 0.0;
  for (int i = 0; i < 9; ++i) {
    sum += f[i];
    jr += EX9[i] * f[i];
    jz += EZ9[i] * f[i];
  }
  for (int i = 0; i < 5; ++i) tsum += g[i];
  *T = tsum;                    /* Eq. (38) */
  double rh = sum / r;          /* Eq. (26) */
  *rho = rh;
  double Gr, Gz;
  body_accel(s, tsum, &Gr, &Gz);
  /* Eq. (29) */
  double vr = (jr + 0.5 * DT * r * phi * rh * Gr + 0.5 * DT * rh * CS2) / rh;
  double vz = (jz + 0.5 * DT * r * phi * rh * Gz) / rh;
  /* Eq. (30) */
  double lr0 = 0.5 * ((r * r + CS2 * (s->tau_nu - 0.5) * DT * DT) / r +
                      r * phi * 0.5 * DT * s->nu / K);
  double lz0 = 0.5 * ((r * r) / r + r * phi * 0.5 * DT * s->nu / K);
  double l1 = r * phi * 0.5 * DT * Fphi / sqrt(K);
  double vmag = sqrt(vr * vr + vz * vz);
  /* Eq. (28) */
  *ur = vr / (lr0 + sqrt(lr0 * lr0 + l1 * vmag));
  *uz = vz / (lz0 + sqrt(lz0 * lz0 + l1 * vmag));
}

/* Eq. (21) then Eq. (22): MRT collision in moment space. */
static void mrt_collide(const orc_state* s, double r, double phi, double rho, double ur,
                        double uz, double Fr, double Fz, double ar, const double* f,
                        double* fout) {
  double m[9], meq[9], S[9], mp[9];
  matvec9(MM, f, m);                       /* Eq. (16) */
  eq_moments(r, rho, ur, uz, phi, meq);    /* Eqs. (19)-(20) */
  source_moments(s->p.src_printed, r, rho, ur, uz, phi, Fr, Fz, ar, S); /* Eq. (24) */
  for (int k = 0; k < 9; ++k)
    mp[k] = m[k] - s->lam[k] * (m[k] - meq[k]) + DT * (1.0 - 0.5 * s->lam[k]) * S[k];
  matvec9(s->Minv, mp, fout);              /* Eq. (22) */
}

/* Eq. (35): temperature equilibrium. */
static double g_eq(int i, double T, double ur, double uz) {
  double eu = EX5[i] * ur + EZ5[i] * uz;
  return W5[i] * T * (1.0 + eu / CST2);
}

/* Eq. (33) with the direction-dependent rate given after it, Eq. (37) source. */
static void thermal_collide(const orc_state* s, double r, double T, double ur, double uz,
                            const double* g, double* gout) {
  for (int i = 0; i < 5; ++i) {
    double geq = g_eq(i, T, ur, uz);
    double omega = (1.0 + EX5[i] * s->tau_T * DT / r) / (s->tau_T + 0.5);
    double psi = -(ur / r) * geq;
    gout[i] = g[i] - omega * (g[i] - geq) + DT * psi;
  }
}

/* ---- geometry ------------------------------------------------------------- */

static uint8_t node_mask(const orc_params* p, int j, int k) {
  uint8_t m = 0;
  if (p->side_rmin == SIDE_WALL && j == 0) m |= MASK_RMIN;
  if (p->side_rmax == SIDE_WALL && j == p->nr - 1) m |= MASK_RMAX;
  const int zb = p->side_z == SIDE_WALL || p->side_z == SIDE_FLOW;
  if (zb && k == 0) m |= MASK_ZMIN;
  if (zb && k == p->nz - 1) m |= MASK_ZMAX;
  if (p->side_rmin == SIDE_AXIS && j == 0) m |= MASK_AXISROW;
  return m;
}

static int is_boundary(uint8_t m) { return (m & 15) != 0; }

/* Fluid neighbour that supplies a wall node's non-equilibrium part (R2). */
static void owner_of(const orc_params* p, uint8_t m, int j, int k, int* jb, int* kb) {
  *jb = j + ((m & MASK_RMIN) ? 1 : 0) - ((m & MASK_RMAX) ? 1 : 0);
  *kb = k + ((m & MASK_ZMIN) ? 1 : 0) - ((m & MASK_ZMAX) ? 1 : 0);
  (void)p;
}

/* Does wall node (mask m, column k) take the flux condition of R9?  *q gets q'/k. */
static int flux_node(const orc_params* p, uint8_t m, int k, double* q) {
  if ((m & MASK_RMIN) && p->therm_rmin == THERM_FIXED) return 0;
  if ((m & MASK_RMAX) && p->therm_rmax == THERM_FIXED) return 0;
  if ((m & (MASK_ZMIN | MASK_ZMAX)) && p->therm_z == THERM_FIXED) return 0;
  if (!(p->flux_zlo <= k && k <= p->flux_zhi)) return 0;
  if ((m & MASK_RMIN) && p->therm_rmin == THERM_FLUX) { *q = p->flux_rmin; return 1; }
  if ((m & MASK_RMAX) && p->therm_rmax == THERM_FLUX) { *q = p->flux_rmax; return 1; }
  return 0;
}

/* Wall temperature (R2, R9). */
static double wall_temperature(const orc_params* p, uint8_t m, int k, double T_owner) {
  double q;
  if ((m & MASK_RMIN) && p->therm_rmin == THERM_FIXED) return p->T_rmin;
  if ((m & MASK_RMAX) && p->therm_rmax == THERM_FIXED) return p->T_rmax;
  if ((m & MASK_ZMIN) && p->therm_z == THERM_FIXED) return p->T_zmin;
  if ((m & MASK_ZMAX) && p->therm_z == THERM_FIXED && p->side_z != SIDE_FLOW) return p->T_zmax;
  if (flux_node(p, m, k, &q)) return T_owner + q * 1.0; /* q'/k times the spacing to B */
  return T_owner;                                       /* adiabatic wall, outlet (R12) */
}

/* Density and velocity of a boundary node (R2, R12) from its owner's values. */
static void boundary_flow(const orc_params* p, uint8_t m, double rho_B, double ur_B, double uz_B,
                          double* rho, double* ur, double* uz) {
  *rho = rho_B; *ur = 0.0; *uz = 0.0;  /* no-slip wall, and every corner with a radial wall */
  if (p->side_z != SIDE_FLOW || (m & (MASK_RMIN | MASK_RMAX))) return;
  if (m & MASK_ZMIN) { *uz = p->u_in; return; }         /* inlet */
  *rho = 1.0; *ur = ur_B; *uz = uz_B;                   /* outlet */
}

/* ---- state ---------------------------------------------------------------- */

static const char* g_err = "";
const char* orc_last_error(void) { return g_err; }

static double kappa(double ph) { return ph * ph * ph / ((1.0 - ph) * (1.0 - ph)); }

/* Derived constants: Eq. (31), Eq. (39), Eq. (9), Eq. (23) with the rates of Sec. 4. */
static int derive(orc_state* s) {
  const orc_params* p = &s->p;
  const double cs = sqrt(CS2);
  if (p->tau_nu > 0.0) {
    s->tau_nu = p->tau_nu;
  } else {
    if (!(p->Ra > 0.0)) { g_err = "tau_nu not given and Ra <= 0"; return -1; }
    s->tau_nu = 0.5 + p->Ma * p->J * p->L * sqrt(p->Pr) / (cs * DT * sqrt(p->Ra)); /* Eq. (39) */
  }
  s->tau_T = CS2 * p->lambda * (s->tau_nu - 0.5) / (CST2 * p->J * p->Pr); /* Eq. (39) */
  s->nu_e = CS2 * (s->tau_nu - 0.5) * DT; /* Eq. (31) */
  s->nu = s->nu_e / p->J;                 /* J = nu_e / nu, Eq. (9) */
  s->K_ref = p->Da * p->L * p->L;         /* Da = K / L^2, Eq. (9) */
  double dT = p->delta_T != 0.0 ? p->delta_T : (p->T_rmin - p->T_rmax);
  if (p->Ra > 0.0) {
    double U = p->Ma * cs;                /* Ma = U / c_s */
    double gbdT = U * U / p->L;           /* U = sqrt(g beta dT L) */
    if (dT == 0.0) { g_err = "buoyancy needs a nonzero temperature difference"; return -1; }
    s->gbeta = gbdT / dT;
  } else {
    s->gbeta = 0.0;
  }
  double snu = p->s_nu > 0.0 ? p->s_nu : 1.0 / s->tau_nu;
  double lam[9] = {1.0, p->s_e, p->s_eps, p->s_j, p->s_q, p->s_j, p->s_q, snu, snu}; /* Eq. (23) */
  memcpy(s->lam, lam, sizeof lam);
  if (invert9(MM, s->Minv) != 0) { g_err = "M is singular"; return -1; }
  return 0;
}

void orc_destroy(orc_state* s) {
  if (!s) return;
  free(s->r); free(s->phi); free(s->K); free(s->Fphi);
  free(s->f); free(s->g); free(s->fp); free(s->gp); free(s->fn); free(s->gn);
  free(s->rho); free(s->ur); free(s->uz); free(s->T);
  free(s->pur); free(s->puz); free(s->pT); free(s->mask);
  free(s);
}

static void compute_all_macros(orc_state* s);

/*
 * Create a lattice.  phi_field ([nz][nr], r fastest) may be NULL for uniform
 * porosity.  init ([3][nz][nr]: u_z, u_r, T) may be NULL: then u = 0 and
 * T = T_init.  Populations start as in reading R8 with rho = 1:
 * f = M^{-1} (m^eq - S/2) (Eqs. 19-20, 24), g = g^eq (Eq. 35).
 */
orc_state* orc_create(const orc_params* p, const double* phi_field, const double* init) {
  const int nr = p->nr, nz = p->nz;
  if (nr < 3 || nz < 1) { g_err = "grid too small"; return NULL; }
  if (p->side_z == SIDE_WALL && nz < 3) { g_err = "axial walls need nz >= 3"; return NULL; }
  if (p->side_rmax == SIDE_AXIS) { g_err = "the axis can only be at r_min"; return NULL; }
  if (p->side_rmin == SIDE_AXIS && p->r0 != 0.5) { g_err = "axis needs r0 = 1/2"; return NULL; }
  if ((p->side_rmin == SIDE_PERIODIC) != (p->side_rmax == SIDE_PERIODIC)) {
    g_err = "radial periodicity must be on both sides"; return NULL;
  }
  if (!(p->r0 > 0.0)) { g_err = "r0 must be positive"; return NULL; }
  if (p->therm_z == THERM_FLUX) { g_err = "flux walls are radial only"; return NULL; }
  if (p->side_rmin == SIDE_FLOW || p->side_rmax == SIDE_FLOW) {
    g_err = "inlet and outlet are axial only"; return NULL;
  }
  if (p->side_z == SIDE_FLOW && nz < 3) { g_err = "inlet and outlet need nz >= 3"; return NULL; }
  orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
  s->p = *p;
  if (derive(s) != 0) { free(s); return NULL; }
  s->nr = nr; s->nz = nz; s->n = nr * nz;
  const int n = s->n;
  s->r = malloc(sizeof(double) * nr);
  s->phi = malloc(sizeof(double) * n); s->K = malloc(sizeof(double) * n);
  s->Fphi = malloc(sizeof(double) * n);
  s->f = malloc(sizeof(double) * 9 * n); s->g = malloc(sizeof(double) * 5 * n);
  s->fp = malloc(sizeof(double) * 9 * n); s->gp = malloc(sizeof(double) * 5 * n);
  s->fn = malloc(sizeof(double) * 9 * n); s->gn = malloc(sizeof(double) * 5 * n);
  s->rho = malloc(sizeof(double) * n); s->ur = malloc(sizeof(double) * n);
  s->uz = malloc(sizeof(double) * n); s->T = malloc(sizeof(double) * n);
  s->pur = malloc(sizeof(double) * n); s->puz = malloc(sizeof(double) * n);
  s->pT = malloc(sizeof(double) * n);
  s->mask = malloc(n);
  for (int j = 0; j < nr; ++j) s->r[j] = p->r0 + j;
  double kref = 0.0;
  if (phi_field) {
    if (!(p->phi > 0.0 && p->phi < 1.0)) { g_err = "a porosity field needs 0 < phi_ref < 1"; orc_destroy(s); return NULL; }
    kref = kappa(p->phi);
  }
  for (int idx = 0; idx < n; ++idx) {
    double ph = phi_field ? phi_field[idx] : p->phi;
    if (!(ph > 0.0 && ph <= 1.0) || (phi_field && !(ph < 1.0))) {
      g_err = "porosity out of range"; orc_destroy(s); return NULL;
    }
    s->phi[idx] = ph;
    s->K[idx] = phi_field ? s->K_ref * kappa(ph) / kref : s->K_ref;  /* Eq. (8), R6 */
    s->Fphi[idx] = p->F_phi >= 0.0 ? p->F_phi : 1.75 / sqrt(150.0 * ph * ph * ph); /* Eq. (8) */
  }
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < nr; ++j) s->mask[k * nr + j] = node_mask(p, j, k);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < nr; ++j) {
      int idx = k * nr + j;
      double uz0 = init ? init[idx] : 0.0;
      double ur0 = init ? init[n + idx] : 0.0;
      double T0 = init ? init[2 * n + idx] : p->T_init;
      double meq[9], S[9], m0[9], Fr, Fz, ar;
      eq_moments(s->r[j], 1.0, ur0, uz0, s->phi[idx], meq);
      total_force(s, s->r[j], s->phi[idx], s->K[idx], s->Fphi[idx], ur0, uz0, T0, &Fr, &Fz, &ar);
      source_moments(p->src_printed, s->r[j], 1.0, ur0, uz0, s->phi[idx], Fr, Fz, ar, S);
      for (int q = 0; q < 9; ++q) m0[q] = meq[q] - 0.5 * DT * S[q];
      matvec9(s->Minv, m0, s->f + 9 * idx);
      for (int i = 0; i < 5; ++i) s->g[5 * idx + i] = g_eq(i, T0, ur0, uz0);
    }
  s->t = 0;
  s->have_prev = 0;
  compute_all_macros(s);
  return s;
}

/* Macroscopic values at time t for every node; wall nodes take R2's values. */
static void compute_all_macros(orc_state* s) {
  const int nr = s->nr, nz = s->nz;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < nr; ++j) {
      int idx = k * nr + j;
      if (is_boundary(s->mask[idx])) continue;
      node_macros(s, s->r[j], s->phi[idx], s->K[idx], s->Fphi[idx], s->f + 9 * idx,
                  s->g + 5 * idx, &s->rho[idx], &s->ur[idx], &s->uz[idx], &s->T[idx]);
    }
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < nr; ++j) {
      int idx = k * nr + j;
      uint8_t m = s->mask[idx];
      if (!is_boundary(m)) continue;
      int jb, kb;
      owner_of(&s->p, m, j, k, &jb, &kb);
      int ib = kb * nr + jb;
      boundary_flow(&s->p, m, s->rho[ib], s->ur[ib], s->uz[ib], &s->rho[idx], &s->ur[idx],
                    &s->uz[idx]);
      s->T[idx] = wall_temperature(&s->p, m, k, s->T[ib]);
    }
}

/* Collision of every node at time t into fp, gp. */
static void collide_all(orc_state* s) {
  const int nr = s->nr, nz = s->nz;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < nr; ++j) {
      int idx = k * nr + j;
      uint8_t m = s->mask[idx];
      double r = s->r[j], phi = s->phi[idx], K = s->K[idx], Fphi = s->Fphi[idx];
      if (!is_boundary(m)) {
        double Fr, Fz, ar;
        total_force(s, r, phi, K, Fphi, s->ur[idx], s->uz[idx], s->T[idx], &Fr, &Fz, &ar);
        mrt_collide(s, r, phi, s->rho[idx], s->ur[idx], s->uz[idx], Fr, Fz, ar, s->f + 9 * idx,
                    s->fp + 9 * idx);
        thermal_collide(s, r, s->T[idx], s->ur[idx], s->uz[idx], s->g + 5 * idx, s->gp + 5 * idx);
        continue;
      }
      /* R2: non-equilibrium extrapolation from the owner B. */
      int jb, kb;
      owner_of(&s->p, m, j, k, &jb, &kb);
      int ib = kb * nr + jb;
      double rB = s->r[jb];
      /* boundary state (R2, R9, R12), set by compute_all_macros */
      double rho = s->rho[idx], urb = s->ur[idx], uzb = s->uz[idx], Tb = s->T[idx];
      double meqb[9], feqb[9], meqB[9], feqB[9], fb[9], gb[5];
      eq_moments(r, rho, urb, uzb, phi, meqb);
      matvec9(s->Minv, meqb, feqb);
      eq_moments(rB, s->rho[ib], s->ur[ib], s->uz[ib], s->phi[ib], meqB);
      matvec9(s->Minv, meqB, feqB);
      for (int i = 0; i < 9; ++i) fb[i] = feqb[i] + (s->f[9 * ib + i] - feqB[i]);
      for (int i = 0; i < 5; ++i)
        gb[i] = g_eq(i, Tb, urb, uzb) +
                (s->g[5 * ib + i] - g_eq(i, s->T[ib], s->ur[ib], s->uz[ib]));
      double Fr, Fz, ar;
      total_force(s, r, phi, K, Fphi, urb, uzb, Tb, &Fr, &Fz, &ar);
      mrt_collide(s, r, phi, rho, urb, uzb, Fr, Fz, ar, fb, s->fp + 9 * idx);
      thermal_collide(s, r, Tb, urb, uzb, gb, s->gp + 5 * idx);
    }
}

static int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Streaming, f_i(x + e_i, t + 1) = f_i^+(x, t) (Eq. 22; Eq. 33 for g). */
static void stream_all(orc_state* s) {
  const int nr = s->nr, nz = s->nz, n = s->n;
  const orc_params* p = &s->p;
  const double nanv = NAN;
  for (int q = 0; q < 9 * n; ++q) s->fn[q] = nanv;  /* entries nobody streams into stay NaN */
  for (int q = 0; q < 5 * n; ++q) s->gn[q] = nanv;
  const int rper = p->side_rmin == SIDE_PERIODIC, zper = p->side_z == SIDE_PERIODIC;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < nr; ++j) {
      int idx = k * nr + j;
      for (int i = 0; i < 9; ++i) {
        int dj = j + EX9[i], dk = k + EZ9[i];
        if (rper) dj = wrap(dj, nr);
        if (zper) dk = wrap(dk, nz);
        if (dj < 0 || dj >= nr || dk < 0 || dk >= nz) continue;
        s->fn[9 * (dk * nr + dj) + i] = s->fp[9 * idx + i];
      }
      for (int i = 0; i < 5; ++i) {
        int dj = j + EX5[i], dk = k + EZ5[i];
        if (rper) dj = wrap(dj, nr);
        if (zper) dk = wrap(dk, nz);
        if (dj < 0 || dj >= nr || dk < 0 || dk >= nz) continue;
        s->gn[5 * (dk * nr + dj) + i] = s->gp[5 * idx + i];
      }
    }
  if (p->side_rmin == SIDE_AXIS) {
    /* R3: populations entering row 0 from the ghost row at r = -1/2. */
    static const int mirror9[9] = {0, 3, 2, 1, 4, 6, 5, 8, 7};
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < 9; ++i) {
        if (EX9[i] != 1) continue;
        int ks = k - EZ9[i];          /* ghost source (-1, ks) mirrors (0, ks) */
        if (zper) ks = wrap(ks, nz);
        if (ks < 0 || ks >= nz) continue;
        s->fn[9 * (k * nr) + i] = -s->fp[9 * (ks * nr) + mirror9[i]];
      }
    for (int k = 0; k < nz; ++k) s->gn[5 * (k * nr) + 1] = s->gp[5 * (k * nr) + 3];
  }
  double* tf = s->f; s->f = s->fn; s->fn = tf;
  double* tg = s->g; s->g = s->gn; s->gn = tg;
}

/* Advance nsteps time steps. */
void orc_step(orc_state* s, int nsteps) {
  for (int it = 0; it < nsteps; ++it) {
    collide_all(s);
    stream_all(s);
    s->t += 1;
    compute_all_macros(s);
  }
}

/* Keep the current velocity and temperature for orc_residual. */
void orc_snapshot(orc_state* s) {
  memcpy(s->pur, s->ur, sizeof(double) * s->n);
  memcpy(s->puz, s->uz, sizeof(double) * s->n);
  memcpy(s->pT, s->T, sizeof(double) * s->n);
  s->t_snap = s->t;
  s->have_prev = 1;
}

long orc_time(const orc_state* s) { return s->t; }

/* Macroscopic fields at time t, [nz][nr]; p = rho c_s^2 / phi (text after Eq. 30). */
void orc_macros(const orc_state* s, double* uz, double* ur, double* p, double* T,
                double* rho, uint8_t* mask) {
  for (int idx = 0; idx < s->n; ++idx) {
    if (uz) uz[idx] = s->uz[idx];
    if (ur) ur[idx] = s->ur[idx];
    if (p) p[idx] = s->rho[idx] * CS2 / s->phi[idx];
    if (T) T[idx] = s->T[idx];
    if (rho) rho[idx] = s->rho[idx];
    if (mask) mask[idx] = s->mask[idx];
  }
}

/*
 * Steady-state residual between the snapshot time t0 and the current time t
 * over the N fluid nodes (the paper gives no criterion): the root-mean-square
 * change per step, sqrt(sum |u^t - u^t0|^2 / N) / (t - t0), scaled by the
 * characteristic velocity U = Ma c_s (text before Eq. 39) in out[0], the same
 * for T scaled by dT in out[1], out[2] = max of both.  Returns -1 without a
 * snapshot or when t = t0.
 */
int orc_residual(const orc_state* s, double* out) {
  if (!s->have_prev || s->t == s->t_snap) return -1;
  const double steps = (double)(s->t - s->t_snap);
  double du = 0, dT = 0;
  long nf = 0;
  for (int idx = 0; idx < s->n; ++idx) {
    if (is_boundary(s->mask[idx])) continue;
    double a = s->ur[idx] - s->pur[idx], b = s->uz[idx] - s->puz[idx];
    du += a * a + b * b;
    double c = s->T[idx] - s->pT[idx];
    dT += c * c;
    nf += 1;
  }
  double U = s->p.Ma > 0.0 ? s->p.Ma * sqrt(CS2) : 1.0;
  double Tc = s->p.delta_T != 0.0 ? fabs(s->p.delta_T) : fabs(s->p.T_rmin - s->p.T_rmax);
  if (Tc == 0.0) Tc = 1.0;
  out[0] = nf ? sqrt(du / nf) / (U * steps) : 0.0;
  out[1] = nf ? sqrt(dT / nf) / (Tc * steps) : 0.0;
  out[2] = out[0] > out[1] ? out[0] : out[1];
  return 0;
}

/*
 * Mean Nusselt numbers on the r_min and r_max walls, Eq. (42):
 * Nu = -(r_w / (H dT)) * integral_0^H (dT/dr)_w dz, with a second-order
 * one-sided radial difference and the trapezoid rule over k = 0..nz-1,
 * H = nz - 1.
 */
void orc_nusselt(const orc_state* s, double* nu_i, double* nu_o) {
  const int nr = s->nr, nz = s->nz;
  const orc_params* p = &s->p;
  double dT = p->delta_T != 0.0 ? p->delta_T : (p->T_rmin - p->T_rmax);
  double H = nz - 1;
  double si = 0.0, so = 0.0;
  for (int k = 0; k < nz; ++k) {
    double c = (k == 0 || k == nz - 1) ? 0.5 : 1.0;
    const double* T = s->T + k * nr;
    double gi = (-3.0 * T[0] + 4.0 * T[1] - T[2]) / 2.0;
    double go = (3.0 * T[nr - 1] - 4.0 * T[nr - 2] + T[nr - 3]) / 2.0;
    si += c * gi;
    so += c * go;
  }
  *nu_i = -(s->r[0] / (H * dT)) * si;
  *nu_o = -(s->r[nr - 1] / (H * dT)) * so;
  /* A flux wall reports the heater mean of Eqs. (43)-(44) instead (R10). */
  for (int side = 0; side < 2; ++side) {
    int therm = side ? p->therm_rmax : p->therm_rmin;
    if (therm != THERM_FLUX) continue;
    int j = side ? nr - 1 : 0;
    double sum = 0.0, q = 0.0;
    int cnt = 0;
    for (int k = 0; k < nz; ++k) {
      int idx = k * nr + j;
      if (!is_boundary(s->mask[idx]) || !flux_node(p, s->mask[idx], k, &q)) continue;
      sum += q * p->L / (s->T[idx] - p->T_ref); /* Eq. (44) */
      cnt += 1;
    }
    double nu = cnt ? sum / cnt : NAN;          /* Eq. (43) */
    if (side) *nu_o = nu; else *nu_i = nu;
  }
}

/*
 * Local pipe Nusselt number and bulk temperature at every column (R13,
 * Eqs. 40-41): area = 0 takes the mixing-cup T_b, area = 1 the area mean as
 * printed.  Needs an axis at r_min and a wall at r_max; returns -1 otherwise.
 */
int orc_pipe_nusselt(const orc_state* s, int area, double* nu, double* Tb) {
  const int nr = s->nr, nz = s->nz;
  if (s->p.side_rmin != SIDE_AXIS || s->p.side_rmax != SIDE_WALL || nr < 3) return -1;
  const double rw = s->r[nr - 1], D = 2.0 * rw;
  for (int k = 0; k < nz; ++k) {
    const double* T = s->T + (long)k * nr;
    const double* u = s->uz + (long)k * nr;
    double num = 0.0, den = 0.0;
    for (int j = 0; j < nr; ++j) {
      /* trapezoid weights over 0, r_0, ..., r_{nr-1}: the first interval
         [0, r_0] adds r_0 / 2 to node 0, each later interval 1/2 to both ends */
      double w = (j == 0 ? 0.5 * s->r[0] : 0.5) + (j < nr - 1 ? 0.5 : 0.0);
      double wu = area ? w : w * u[j];
      num += wu * s->r[j] * T[j];
      den += wu * s->r[j];
    }
    double tb = num / den;                                          /* Eq. (41) */
    double g = (3.0 * T[nr - 1] - 4.0 * T[nr - 2] + T[nr - 3]) / 2.0;
    if (Tb) Tb[k] = tb;
    if (nu) nu[k] = D * g / (T[nr - 1] - tb);                      /* Eq. (40) */
  }
  return 0;
}

/*
 * Stokes stream function (R11) of a u_z field ([nz][nr], rows at r0 + j):
 * psi[k][j] = psi[k][j-1] + (r_{j-1} u_{j-1} + r_j u_j) / 2 (trapezoid rule of
 * the integral of r u_z dr), starting from psi[k][0] = 0 on an r_min wall, or,
 * with axis = 1, from psi[k][0] = r0 (r0 u_0) / 2 (the interval [0, r0], where
 * r u_z vanishes on the axis).  Returns max |psi|.
 */
double orc_stream_function(int nr, int nz, double r0, int axis, const double* uz, double* psi) {
  double mx = 0.0;
  for (int k = 0; k < nz; ++k) {
    const double* u = uz + (long)k * nr;
    double acc = axis ? 0.5 * r0 * (r0 * u[0]) : 0.0;
    if (psi) psi[(long)k * nr] = acc;
    if (fabs(acc) > mx) mx = fabs(acc);
    for (int j = 1; j < nr; ++j) {
      acc += 0.5 * ((r0 + j - 1) * u[j - 1] + (r0 + j) * u[j]);
      if (psi) psi[(long)k * nr + j] = acc;
      if (fabs(acc) > mx) mx = fabs(acc);
    }
  }
  return mx;
}

/* Raw populations, [nz][nr][9] and [nz][nr][5]. */
void orc_get_populations(const orc_state* s, double* f, double* g) {
  if (f) memcpy(f, s->f, sizeof(double) * 9 * s->n);
  if (g) memcpy(g, s->g, sizeof(double) * 5 * s->n);
}
void orc_set_populations(orc_state* s, const double* f, const double* g) {
  if (f) memcpy(s->f, f, sizeof(double) * 9 * s->n);
  if (g) memcpy(s->g, g, sizeof(double) * 5 * s->n);
  compute_all_macros(s);
}

/* Derived constants: tau_nu, tau_T, nu_e, nu, K_ref, g*beta. */
void orc_derived(const orc_state* s, double* out) {
  out[0] = s->tau_nu; out[1] = s->tau_T; out[2] = s->nu_e;
  out[3] = s->nu; out[4] = s->K_ref; out[5] = s->gbeta;
}

/* M (Eq. 18) and the inverse this oracle uses. */
void orc_matrices(const orc_state* s, double* M, double* Minv) {
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      if (M) M[9 * i + j] = MM[i][j];
      if (Minv) Minv[9 * i + j] = s->Minv[i][j];
    }
}

/*
 * One node in isolation, for identity checks: given r, phi, f[9], g[5],
 * returns the macroscopic values (rho, u_r, u_z, T, Ft_r, Ft_z, a_r), the
 * equilibrium moments, the source moments and the post-collision f, g.
 */
void orc_node(const orc_state* s, double r, double phi, const double* f, const double* g,
              double* macro, double* meq, double* S, double* fout, double* gout) {
  double K = s->K_ref;
  if (s->p.phi > 0.0 && s->p.phi < 1.0 && phi != s->p.phi) K = s->K_ref * kappa(phi) / kappa(s->p.phi);
  double Fphi = s->p.F_phi >= 0.0 ? s->p.F_phi : 1.75 / sqrt(150.0 * phi * phi * phi);
  double rho, ur, uz, T, Fr, Fz, ar;
  node_macros(s, r, phi, K, Fphi, f, g, &rho, &ur, &uz, &T);
  total_force(s, r, phi, K, Fphi, ur, uz, T, &Fr, &Fz, &ar);
  if (macro) {
    macro[0] = rho; macro[1] = ur; macro[2] = uz; macro[3] = T; macro[4] = Fr + ar;
    macro[5] = Fz; macro[6] = ar;
  }
  if (meq) eq_moments(r, rho, ur, uz, phi, meq);
  if (S) source_moments(s->p.src_printed, r, rho, ur, uz, phi, Fr, Fz, ar, S);
  if (fout) mrt_collide(s, r, phi, rho, ur, uz, Fr, Fz, ar, f, fout);
  if (gout) thermal_collide(s, r, T, ur, uz, g, gout);
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
