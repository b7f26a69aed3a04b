// Host-side derivation of an instance descriptor from the problem statement:
// Eq. (39) relaxation times, Eq. (31) viscosity, Eq. (9) permeability,
// buoyancy g beta = (Ma c_s)^2 / (L dT) and the porosity coefficients of
// Eqs. (6) and (8).  Device pointers are left null.
#pragma once

#include <cmath>
#include <cstring>
#include <string>

#include "../../include/lbm_axi.h"
#include "lbm_axi_dev.h"

namespace lbmaxi {

inline double kappa(double ph) { return ph * ph * ph / ((1.0 - ph) * (1.0 - ph)); }

// Constants of one instance derived from its problem statement, in FP64:
// tau_nu and tau_T (Eq. 39), the effective viscosity nu_e (Eq. 31), the
// fluid viscosity nu = nu_e / J and the reference permeability K = Da L^2
// (Eq. 9), g beta = (Ma c_s)^2 / (L dT) (0 without buoyancy) and the
// effective thermal diffusivity alpha_e = c_sT^2 tau_T (text after Eq. 38).
struct Derived {
  double tau_nu, tau_T, nu_e, nu, K_ref, gbeta, alpha_e;
};

inline Derived derive(const lbm_axi_params& q) {
  Derived d;
  const double cs = std::sqrt(1.0 / 3.0);
  d.tau_nu = q.tau_nu > 0.0 ? q.tau_nu
                            : 0.5 + q.Ma * q.J * q.L * std::sqrt(q.Pr) / (cs * std::sqrt(q.Ra));  // Eq. (39)
  d.tau_T = (1.0 / 3.0) * q.lambda * (d.tau_nu - 0.5) / (0.2 * q.J * q.Pr);                // Eq. (39)
  d.nu_e = (1.0 / 3.0) * (d.tau_nu - 0.5);                                                  // Eq. (31)
  d.nu = d.nu_e / q.J;  // J = nu_e / nu
  d.K_ref = q.Da * q.L * q.L;  // Da = K / L^2
  const double dT = q.delta_T != 0.0 ? q.delta_T : q.T_rmin - q.T_rmax;
  d.gbeta = (q.Ra > 0.0 && dT != 0.0) ? (q.Ma * cs) * (q.Ma * cs) / q.L / dT : 0.0;  // U = sqrt(g beta dT L)
  d.alpha_e = 0.2 * d.tau_T;
  return d;
}

// Returns LBM_AXI_OK or an error code with a message in err.
inline int describe(const lbm_axi_params& q, bool field, InstDev& D, std::string& err) {
  std::memset(&D, 0, sizeof(D));
  D.nr = q.nr;
  D.nz = q.nz;
  D.stride = (q.nr + 63) / 64 * 64;
  D.plane = (int64_t)D.stride * q.nz;
  D.side_rmin = q.side_rmin;
  D.side_rmax = q.side_rmax;
  D.side_z = q.side_z;
  D.therm_rmin = q.therm_rmin;
  D.therm_rmax = q.therm_rmax;
  D.therm_z = q.therm_z;
  D.src_printed = q.src_printed ? 1 : 0;
  const Derived dv = derive(q);
  const double tau = dv.tau_nu, tauT = dv.tau_T, nu = dv.nu, Kref = dv.K_ref, gbeta = dv.gbeta;
  if (!(tau > 0.5)) {
    err = "tau_nu must exceed 1/2";
    return LBM_AXI_EINVAL;
  }
  const double dT = q.delta_T != 0.0 ? q.delta_T : q.T_rmin - q.T_rmax;
  if (q.Ra > 0.0 && dT == 0.0) {
    err = "buoyancy needs a nonzero temperature difference";
    return LBM_AXI_EINVAL;
  }
  D.r0 = (float)q.r0;
  D.T_ref = (float)q.T_ref;
  D.gbeta = (float)gbeta;
  D.accel_r = (float)q.accel_r;
  D.accel_z = (float)q.accel_z;
  // Temperature storage shift: the start temperature in FP32 (errors then
  // scale with T - T_init), the mid temperature in 16-bit storage (smallest
  // magnitude range).
  const double Ts = q.storage == LBM_STORE_FP32 ? q.T_init : q.T_ref;
  D.T_s = (float)Ts;
  D.az_s = (float)(q.accel_z + gbeta * (Ts - q.T_ref));
  D.c_tau = (float)((1.0 / 3.0) * (tau - 0.5));
  D.s_e = (float)q.s_e;
  D.s_eps = (float)q.s_eps;
  D.s_j = (float)q.s_j;
  D.s_q = (float)q.s_q;
  D.s_nu = (float)(1.0 / tau);
  D.tau_T = (float)tauT;
  D.omc = (float)(1.0 / (tauT + 0.5));
  D.T_rmin = (float)q.T_rmin;
  D.T_rmax = (float)q.T_rmax;
  D.T_zmin = (float)q.T_zmin;
  D.T_zmax = (float)q.T_zmax;
  const double Fphi_u = q.F_phi >= 0.0 ? q.F_phi : 1.75 / std::sqrt(150.0 * q.phi * q.phi * q.phi);
  D.phiu = (float)q.phi;
  D.cD = (float)(q.phi * nu / Kref);
  D.cF = (float)(q.phi * Fphi_u / std::sqrt(Kref));
  if (field) {
    // K(phi) = Kref kappa(phi) / kappa(phi_ref) (Eq. 8 with d_p fixed), so
    // phi nu / K = C1 ((1 - phi) / phi)^2 and, with the Ergun F_phi,
    // phi F_phi / sqrt(K) = C2 (1 - phi) / phi^2; with a constant F_phi it is
    // C3 (1 - phi) / sqrt(phi).
    const double kr = kappa(q.phi);
    D.phi_mode = q.F_phi < 0.0 ? 1 : 2;
    D.C1 = (float)(nu * kr / Kref);
    D.C2 = (float)(1.75 * std::sqrt(kr / (150.0 * Kref)));
    D.C3 = (float)(q.F_phi * std::sqrt(kr / Kref));
  }
  // Isoflux window: columns k with flux_zlo <= k <= flux_zhi (clamped to the grid).
  D.q_rmin = (float)q.flux_rmin;
  D.q_rmax = (float)q.flux_rmax;
  const double klo = std::ceil(q.flux_zlo), khi = std::floor(q.flux_zhi);
  D.qk_lo = klo <= 0.0 ? 0 : (klo >= q.nz ? q.nz : (int32_t)klo);
  D.qk_hi = khi < 0.0 ? -1 : (khi >= q.nz - 1 ? q.nz - 1 : (int32_t)khi);
  D.u_in = (float)q.u_in;
  int shift = q.storage_shift;
  if (q.storage == LBM_STORE_FP16 && shift == 0) shift = 10;
  D.st_scale = q.storage == LBM_STORE_FP32 ? 1.0f : std::ldexp(1.0f, shift);
  D.st_inv = q.storage == LBM_STORE_FP32 ? 1.0f : std::ldexp(1.0f, -shift);
  return LBM_AXI_OK;
}

}  // namespace lbmaxi
