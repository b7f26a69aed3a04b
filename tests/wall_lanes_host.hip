// Host build of the step kernel's node code (FP32 storage) for the CPU test
// of the radial wall lanes (tests/test_wall_lanes_host.py).  Each fluid row
// runs as one wave of the step kernel does: every node of the row loads its
// populations before any node of the row stores, so a wall lane sees its
// owner's populations as they were before the step, and its stores into the
// wall column follow its owner's loads.  wlmode 1 runs the wall lanes, 0 the
// owners' wall-node pass.  The padding columns of every row hold a sentinel
// that no store may change.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "../paper_1409_5929_amd/csrc/lbm_axi_desc.h"
#include "../paper_1409_5929_amd/csrc/lbm_axi_dev.h"

using namespace lbmaxi;

namespace {

struct Lane {
  int j, wl;
  RowC R;
  float s[9], t[5], ph;
};

template <bool ODD>
void step_row(const InstDev& D, int k, int wlmode, std::vector<Lane>& lanes) {
  const FieldOut none{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  lanes.clear();
  for (int jt = 0; jt < D.nr; ++jt) {
    const int wl = (D.side_rmin == SIDE_WALL && jt == 0) ? 1 : (D.side_rmax == SIDE_WALL && jt == D.nr - 1) ? -1 : 0;
    const bool wall = (D.side_rmin == SIDE_WALL && jt == 0) || (D.side_rmax == SIDE_WALL && jt == D.nr - 1);
    if (wall && (!wlmode || (wl < 0 && !wall_lane_rmax(D)))) continue;  // the owner takes it
    Lane L;
    L.wl = wlmode ? wl : 0;
    L.j = jt + L.wl;
    L.R = make_row(D, L.j);
    node_load<float, ODD, false>(D, L.R, L.j, k, L.s, L.t, L.ph);
    lanes.push_back(L);
  }
  for (Lane& L : lanes) {
    if (wlmode)
      node_update_loaded<float, ODD, MODE_STEP, false, true>(D, L.R, L.j, k, 0, none, 0u, L.s, L.t, L.ph, L.wl);
    else
      node_update_loaded<float, ODD, MODE_STEP, false, false>(D, L.R, L.j, k, 0, none, 0u, L.s, L.t, L.ph, 0);
  }
}

}  // namespace

// n steps from the start fields init (u_z, u_r, T, each nz x nr; null: rest
// at T_init); the fields of the fluid nodes after them (wall nodes 0).
// Returns 0, -1 for a bad problem, -2 when a padding sentinel changed.
extern "C" int host_wall_lane_steps(const lbm_axi_params* p, const float* phi_field, const float* init,
                                    int nsteps, int wlmode, float* uz, float* ur, float* drho, float* T) {
  InstDev D;
  std::string err;
  if (describe(*p, phi_field != nullptr, D, err)) return -1;
  std::vector<float> pop((size_t)14 * D.plane, 0.0f), phi;
  D.pop = pop.data();
  D.g0 = pop.data() + 9 * D.plane;
  if (phi_field) {
    phi.assign(D.plane, (float)p->phi);
    for (int k = 0; k < p->nz; ++k) memcpy(&phi[(size_t)k * D.stride], phi_field + (size_t)k * p->nr, 4 * p->nr);
    D.phi = phi.data();
  }
  const size_t pl = (size_t)D.nr * D.nz;
  for (int k = 0; k < D.nz; ++k)
    for (int j = 0; j < D.nr; ++j) {
      const size_t o = (size_t)k * D.nr + j;
      if (init) init_node<float>(D, j, k, init[o], init[pl + o], init[2 * pl + o]);
      else init_node<float>(D, j, k, 0.0f, 0.0f, (float)p->T_init);
    }
  const float SENTINEL = 12345.0f;
  for (int q = 0; q < 14; ++q)
    for (int k = 0; k < D.nz; ++k)
      for (int j = D.nr; j < D.stride; ++j) pop[(size_t)q * D.plane + (size_t)k * D.stride + j] = SENTINEL;
  std::vector<Lane> lanes;
  for (int n = 0; n < nsteps; ++n)
    for (int k = 0; k < D.nz; ++k) {
      if (z_bounded(D) && (k == 0 || k == D.nz - 1)) continue;
      if (n & 1) step_row<true>(D, k, wlmode, lanes);
      else step_row<false>(D, k, wlmode, lanes);
    }
  for (int q = 0; q < 14; ++q)
    for (int k = 0; k < D.nz; ++k)
      for (int j = D.nr; j < D.stride; ++j)
        if (pop[(size_t)q * D.plane + (size_t)k * D.stride + j] != SENTINEL) return -2;
  const FieldOut fo{uz, ur, nullptr, T, nullptr, drho};
  for (int j = 0; j < D.nr; ++j) {
    if ((D.side_rmin == SIDE_WALL && j == 0) || (D.side_rmax == SIDE_WALL && j == D.nr - 1)) continue;
    const RowC R = make_row(D, j);
    for (int k = 0; k < D.nz; ++k) {
      if (z_bounded(D) && (k == 0 || k == D.nz - 1)) continue;
      if (nsteps & 1) node_update<float, true, MODE_FIELDS>(D, R, j, k, 0, fo, 0u);
      else node_update<float, false, MODE_FIELDS>(D, R, j, k, 0, fo, 0u);
    }
  }
  return 0;
}
