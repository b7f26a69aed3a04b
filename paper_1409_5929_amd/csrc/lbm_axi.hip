// lbm_axi: C-ABI library of the axisymmetric MRT lattice Boltzmann model for
// thermal flow in porous media (Liu, He, Li, arXiv:1409.5929) on gfx950.
//
// Kernels
//   k_step     fused D2Q9-MRT + D2Q5 collide-stream, AA pattern, in place
//              (lbm_axi_dev.h); optionally writes u_z, u_r, T for the check
//   k_resid    FP64 partial sums of the residual and of the Eq. (42) wall
//              integrals, or of the heater sums of Eqs. (43)-(44) on an
//              isoflux wall (wave shuffles, then LDS across the block's waves)
//   k_final    per-instance reduction of the partials, run-state update
//   k_init     start state
//   k_convert  storage conversion (FP32 / FP16 / BF16) of one instance
//   k_setclock device clock read by captured step graphs
//   k_psi, k_absmax  Stokes stream function of one instance and its largest magnitude
//   k_pipe_nu  local pipe Nusselt number and bulk temperature of one instance
//   k_step<MODE_FIELDS>  macroscopic fields of one instance (no population writes)
//
// Launch geometry: blocks of 64 x 4 threads; lanes run along r (coalesced
// rows), the 4 waves take interleaved z rows, and each thread walks kz rows
// so that its per-radius constants are computed once.  Tiles of all running
// instances form one list; block b takes tile (b % 8) * ceil(T / 8) + b / 8,
// so that each of the 8 XCDs (blocks are dealt to XCDs round-robin) sweeps a
// contiguous band of rows and neighbouring tiles share its L2.
//
// Stepping: runs of plain steps replay a captured HIP graph (kernels only);
// steps that fall on a check, and every step while launches are timed, are
// launched one by one.  Both give identical results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lbm_axi.h"
#include "lbm_axi_desc.h"
#include "lbm_axi_dev.h"
#include "lbm_axi_kernels.h"

using namespace lbmaxi;

namespace {

constexpr int RB = 256;  // threads of the reduction kernels

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(LBM_AXI_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

struct DevResult {
  double res, res_u, res_T, nu_i, nu_o, u_rms;
  long long t_check, t_stop;  // handle time levels (t_stop: level at which the run stopped)
  long long t_off;  // handle steps the instance sat out while stopped (even); its own
                    // time level is the handle's minus t_off
  long long t_arm;  // first check whose comparison spans steps the instance took
  // previous check, for the tail extrapolation: residual parts, Nusselt
  // numbers and their change over the interval before it
  double ru_prev, rT_prev, nu_i_prev, nu_o_prev, dnu_i_prev, dnu_o_prev;
};

struct ResTile {
  int inst, k0, k1, pad;
};

// Scratch of lbm_axi_stream_function_static, for callers that cannot
// allocate: the u_z field of one instance (at most SCRATCH_NODES floats) and
// its per-column maxima (at most SCRATCH_COLS doubles).  Each device holds its
// own copy for the life of the process; host code must use the per-device
// address from hipGetSymbolAddress (scratch_address), never the array's name.
constexpr int64_t SCRATCH_NODES = int64_t(1) << 23;
constexpr int64_t SCRATCH_COLS = int64_t(1) << 16;
constexpr int MAX_DEVICES = 64;
__device__ __align__(256) unsigned char scratch[SCRATCH_NODES * 4 + SCRATCH_COLS * 8];

std::mutex g_scratch_mu;
void* g_scratch[MAX_DEVICES] = {};

}  // namespace

struct lbm_axi {
  int device = 0;               // HIP device the handle was created on
  void* scratch = nullptr;      // that device's copy of the static scratch array
  int n_inst = 0;
  int storage = 0;
  int check = 0;
  int kz = 4;
  bool tiles_set = false;       // launch shape chosen by lbm_axi_set_tiles / lbm_axi_autotune
  int lds_bytes = 0;            // dynamic LDS per step block (caps blocks per CU)
  int lds_per_cu = 0;           // LDS of one compute unit
  int lds_per_block = 0;        // largest LDS one block may reserve
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<lbm_axi_params> prm;
  std::vector<InstDev> hdesc;
  InstDev* ddesc = nullptr;
  std::vector<void*> allocs;
  int4* dtiles = nullptr;       // XCD-ordered tiles of all instances, even steps (own allocation)
  int ntiles_launch = 0;
  int4* dtiles_odd = nullptr;   // the same for odd steps, strips of kz_odd nodes (own allocation)
  int ntiles_odd = 0;
  int kz_odd = 1;
  int4* dtiles_plain = nullptr; // tiles in instance order (own allocation)
  std::vector<int> tile_first, tile_count;
  ResTile* drt = nullptr;
  int nrt = 0;
  double* dpart = nullptr;      // [nrt][6]
  double* dtol = nullptr;       // per-instance tolerance
  double* dtail = nullptr;      // per-instance tail tolerance (0: none)
  double* dnus = nullptr;       // per instance: r_w / (H dT) of both walls, 1 / (Ma c_s), 1 / dT
  long long* dmx = nullptr;     // per-instance max_steps
  int* dstatus = nullptr;
  DevResult* dres = nullptr;
  int* dfirst = nullptr;        // per-instance first reduction tile and count
  long long t = 0;              // global time level
  size_t bytes = 0;
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double timed_ms = 0.0;
  long long timed_launches = 0;
  std::vector<char> active;     // instances in the launch list (empty: all)
  bool buf = false;             // step kernels use buffer addressing (all arrays below 4 GiB)
  bool wall_lanes = false;      // step kernels compute radial wall nodes on their own lanes
  long long* dclk = nullptr;    // device clock of captured step graphs
  int graph_steps = 32;         // steps per captured graph (0: no graphs)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

// ---- kernels ------------------------------------------------------------------


// Plain in-place read+write stream over n 16-byte words (bits XORed with key).
__global__ __launch_bounds__(RB) void k_stream_rw(uint4* __restrict__ p, int64_t n, uint32_t key) {
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += stride) {
    uint4 v = p[i];
    v.x ^= key;
    v.y ^= key;
    v.z ^= key;
    v.w ^= key;
    p[i] = v;
  }
}

// The same with lanes of sizeof(T) bytes (2, 4, 8 or 16): the lane width
// probe.
__device__ inline uint16_t lane_xor(uint16_t v, uint32_t k) { return (uint16_t)(v ^ k); }
__device__ inline uint32_t lane_xor(uint32_t v, uint32_t k) { return v ^ k; }
__device__ inline uint2 lane_xor(uint2 v, uint32_t k) { return make_uint2(v.x ^ k, v.y ^ k); }
__device__ inline uint4 lane_xor(uint4 v, uint32_t k) { return make_uint4(v.x ^ k, v.y ^ k, v.z ^ k, v.w ^ k); }
template <typename T>
__global__ __launch_bounds__(RB) void k_stream_lane(T* __restrict__ p, int64_t n, uint32_t key) {
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += stride) p[i] = lane_xor(p[i], key);
}

// Sets the device clock read by captured step graphs.
__global__ void k_setclock(long long* clk, long long t) {
  if (threadIdx.x == 0) *clk = t;
}

// Storage conversion of one instance: every slot keeps its deviation; the
// temperature slots move from the shift T_s of the source storage to that of
// the target (g_i - wt_i T_s).  Walls' slots are converted like any other.
template <typename Si, typename So>
__global__ __launch_bounds__(RB) void k_convert(const InstDev Di, const InstDev Do) {
  const int64_t o = (int64_t)blockIdx.x * RB + threadIdx.x;
  if (o >= Di.plane || (int)(o % Di.stride) >= Di.nr) return;
  const Si* P = (const Si*)Di.pop;
  So* Q = (So*)Do.pop;
  const int64_t pl = Di.plane;
  const float dT = Di.T_s - Do.T_s;
#pragma unroll
  for (int q = 0; q < 9; ++q)
    Store<So>::st(Q, slot_elem<So>(q, o, pl), Store<Si>::ld(P, slot_elem<Si>(q, o, pl), Di.st_inv),
                  Do.st_scale);
  const float g0 = Di.g0[o] + WT0 * dT;
#pragma unroll
  for (int q = 1; q < 5; ++q)
    Store<So>::st(Q, slot_elem<So>(9 + q, o, pl),
                  Store<Si>::ld(P, slot_elem<Si>(9 + q, o, pl), Di.st_inv) + WT1 * dT, Do.st_scale);
  Do.g0[o] = g0;  // after the loads: in FP32 both g_0 planes may be plane 9 of one array
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// FP64 partial sums over fluid nodes of the rows [k0, k1) of one instance:
// |du|^2, node count, dT^2, |u|^2, and the Eq. (42) integrands on both walls.
__global__ __launch_bounds__(RB) void k_resid(const InstDev* __restrict__ descs,
                                              const ResTile* __restrict__ rts, int cur,
                                              const int* __restrict__ status,
                                              double* __restrict__ part) {
  const ResTile rt = rts[blockIdx.x];
  if (status[rt.inst] != RUN) return;  // k_final skips stopped instances
  const InstDev D = descs[rt.inst];
  const float* cu = cur ? D.mac[1] : D.mac[0];
  const float* pv = cur ? D.mac[0] : D.mac[1];
  const int64_t pl = D.plane;
  double a[6] = {0, 0, 0, 0, 0, 0};
  for (int k = rt.k0; k < rt.k1; ++k) {
    const double ck = (k == 0 || k == D.nz - 1) ? 0.5 : 1.0;
    for (int j = threadIdx.x; j < D.nr; j += RB) {
      const int64_t o = (int64_t)k * D.stride + j;
      if (!is_boundary(D, j, k)) {
        const double uz = cu[o], ur = cu[pl + o], T = cu[2 * pl + o];
        const double duz = uz - (double)pv[o], dur = ur - (double)pv[pl + o];
        const double dT = T - (double)pv[2 * pl + o];
        (void)T;
        a[0] += duz * duz + dur * dur;
        a[1] += 1.0;
        a[2] += dT * dT;
        a[3] += uz * uz + ur * ur;
      }
      // Walls: the Eq. (42) integrand, or on an isoflux wall 1 / (T_h - T_0) of
      // each heated node for the heater mean of Eqs. (43)-(44).
      float q;
      if (j == 0 && D.nr >= 3) {
        if (D.therm_rmin != THERM_FLUX) {
          const double g = (-3.0 * cu[2 * pl + o] + 4.0 * cu[2 * pl + o + 1] - cu[2 * pl + o + 2]) * 0.5;
          a[4] += ck * g;
        } else if (is_boundary(D, j, k) && flux_node(D, node_mask(D, j, k), k, q)) {
          a[4] += 1.0 / ((double)cu[2 * pl + o] - (double)D.T_ref);
        }
      }
      if (j == D.nr - 1 && D.nr >= 3) {
        if (D.therm_rmax != THERM_FLUX) {
          const double g = (3.0 * cu[2 * pl + o] - 4.0 * cu[2 * pl + o - 1] + cu[2 * pl + o - 2]) * 0.5;
          a[5] += ck * g;
        } else if (is_boundary(D, j, k) && flux_node(D, node_mask(D, j, k), k, q)) {
          a[5] += 1.0 / ((double)cu[2 * pl + o] - (double)D.T_ref);
        }
      }
    }
  }
  __shared__ double sh[RB / 64][6];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int q = 0; q < 6; ++q) {
    const double v = wave_sum(a[q]);
    if (lane == 0) sh[w][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = 0.0;
    for (int i = 0; i < RB / 64; ++i) v += sh[i][threadIdx.x];
    part[(int64_t)blockIdx.x * 6 + threadIdx.x] = v;
  }
}

// Per running instance (one block each): sum its partials in a fixed order,
// form the residual (root-mean-square change of u and T over the fluid nodes
// since the previous check, per step, scaled by Ma c_s and dT) and the
// Nusselt numbers, update the run state.  A stopped instance keeps the
// results of the check at which it stopped.  A check before t_arm (the first
// one after a restart) compares with a check buffer the instance did not
// write one interval earlier: it records the Nusselt numbers only.
__global__ __launch_bounds__(RB) void k_final(const int* __restrict__ first,
                                              const double* __restrict__ part, long long t,
                                              double per_step, const double* __restrict__ tol,
                                              const double* __restrict__ tail_tol,
                                              const long long* __restrict__ max_steps,
                                              const double* __restrict__ nu_scale,
                                              int* __restrict__ status,
                                              DevResult* __restrict__ out) {
  const int inst = blockIdx.x;
  if (status[inst] != RUN) return;  // uniform across the block
  double a[6] = {0, 0, 0, 0, 0, 0};
  const int b0 = first[2 * inst], nb = first[2 * inst + 1];
  for (int b = b0 + (int)threadIdx.x; b < b0 + nb; b += RB)
    for (int q = 0; q < 6; ++q) a[q] += part[(int64_t)b * 6 + q];
  __shared__ double sh[RB / 64][6];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int q = 0; q < 6; ++q) {
    const double v = wave_sum(a[q]);
    if (lane == 0) sh[w][q] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int q = 0; q < 6; ++q) {
    double v = 0.0;
    for (int i = 0; i < RB / 64; ++i) v += sh[i][q];
    a[q] = v;
  }
  const double nf = a[1] > 0.0 ? a[1] : 1.0;
  const double ru = sqrt(a[0] / nf) * nu_scale[4 * inst + 2] * per_step;
  const double rT = sqrt(a[2] / nf) * nu_scale[4 * inst + 3] * per_step;
  double res = ru > rT ? ru : rT;
  if (ru != ru || rT != rT) res = ru + rT;  // NaN propagates
  DevResult r = out[inst];
  r.res = res;
  r.res_u = ru;
  r.res_T = rT;
  r.nu_i = -nu_scale[4 * inst] * a[4];
  r.nu_o = -nu_scale[4 * inst + 1] * a[5];
  r.u_rms = sqrt(a[3] / nf);
  r.t_check = t;
  const double nu_i_old = r.nu_i_prev, nu_o_old = r.nu_o_prev;
  r.nu_i_prev = r.nu_i;
  r.nu_o_prev = r.nu_o;
  if (t < r.t_arm) {
    r.res = r.res_u = r.res_T = r.ru_prev = r.rT_prev = HUGE_VAL;
    r.dnu_i_prev = r.dnu_o_prev = HUGE_VAL;
    out[inst] = r;
    return;
  }
  // Geometric tail of the changes still to come (when asked for), for each
  // of u, T (rates: the sum of the future interval changes is
  // rate rho / (1 - rho) / per_step with rho the ratio of successive rates)
  // and the two wall Nusselt numbers (relative change over the interval;
  // changes below 1e-7 of Nu, its resolution from FP32 fields, count as 0).
  bool tail_ok = true;
  const double dni = fabs(r.nu_i - nu_i_old), dno = fabs(r.nu_o - nu_o_old);
  if (tail_tol[inst] > 0.0) {
    const double tt = tail_tol[inst];
    auto tail = [](double now, double before) {  // unknown before (+inf): no estimate yet
      const double rho = before > 0.0 && before < HUGE_VAL ? now / before : HUGE_VAL;
      return rho < 1.0 ? now * rho / (1.0 - rho) : HUGE_VAL;
    };
    tail_ok = tail(ru, r.ru_prev) / per_step <= tt || ru == 0.0;
    tail_ok = tail_ok && (tail(rT, r.rT_prev) / per_step <= tt || rT == 0.0);
    const double ni = fabs(r.nu_i), no = fabs(r.nu_o);
    if (isfinite(r.nu_i) && ni > 0.0 && dni > 1e-7 * ni) tail_ok = tail_ok && tail(dni, r.dnu_i_prev) <= tt * ni;
    if (isfinite(r.nu_o) && no > 0.0 && dno > 1e-7 * no) tail_ok = tail_ok && tail(dno, r.dnu_o_prev) <= tt * no;
  }
  r.ru_prev = ru;
  r.rT_prev = rT;
  r.dnu_i_prev = dni;
  r.dnu_o_prev = dno;
  int st = RUN;
  if (!isfinite(res)) st = DIVERGED;
  else if (res == 0.0 || (res <= tol[inst] && tail_ok)) st = CONVERGED;
  else if (max_steps[inst] > 0 && t + 1 - r.t_off >= max_steps[inst]) st = STALLED;
  if (st != RUN) {
    r.t_stop = t + 1;
    status[inst] = st;
  }
  out[inst] = r;
}

// Stokes stream function of a u_z field [nz][nr] with rows at r0 + j, zero
// on the r_min wall, or with axis = 1 on the axis r = 0 (row 0 then holds
// r0 (r0 u_0) / 2, the trapezoid over [0, r0]): one wave per column k scans the
// trapezoid terms (r_{j-1} u_{j-1} + r_j u_j) / 2 along r in FP64, 64 rows at a
// time, and writes psi (if non-null) and colmax[k] = max_j |psi[k][j]|.
__global__ __launch_bounds__(RB) void k_psi(const float* __restrict__ uz, int nr, int nz, double r0,
                                            int axis, float* __restrict__ psi,
                                            double* __restrict__ colmax) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (RB / 64) + (threadIdx.x >> 6);
  if (k >= nz) return;  // whole waves leave together
  const float* u = uz + (int64_t)k * nr;
  double carry = axis ? 0.5 * r0 * (r0 * (double)u[0]) : 0.0, mx = 0.0;
  for (int j0 = 0; j0 < nr; j0 += 64) {
    const int j = j0 + lane;
    double t = 0.0;
    if (j >= 1 && j < nr) t = 0.5 * ((r0 + (j - 1)) * (double)u[j - 1] + (r0 + j) * (double)u[j]);
    for (int off = 1; off < 64; off <<= 1) {
      const double y = __shfl_up(t, off, 64);
      if (lane >= off) t += y;
    }
    const double v = carry + t;
    if (j < nr) {
      if (psi) psi[(int64_t)k * nr + j] = (float)v;
      mx = fmax(mx, fabs(v));
    }
    carry = __shfl(v, 63, 64);
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) colmax[k] = mx;
}

// Local pipe Nusselt number (Eq. 40) and bulk temperature of one column per
// wave, in FP64 from the FP32 fields [nz][nr] (rows at r0 + j, wall row
// nr-1): T_b = sum v_j r_j T_j / sum v_j r_j with v_j = w_j u_z,j (mixing cup)
// or v_j = w_j (area mean, Eq. 41 as printed) and the trapezoid weights w_j
// over the points 0, r_0, ..., r_{nr-1} (the integrands vanish on the axis);
// Nu = 2 r_w (dT/dr)_w / (T_w - T_b) with the second-order one-sided wall
// gradient.
__global__ __launch_bounds__(RB) void k_pipe_nu(const float* __restrict__ T,
                                                const float* __restrict__ U, int area, int nr,
                                                int nz, double r0, double* __restrict__ nu,
                                                double* __restrict__ tb) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (RB / 64) + (threadIdx.x >> 6);
  if (k >= nz) return;  // whole waves leave together
  const float* t = T + (int64_t)k * nr;
  const float* u = U + (int64_t)k * nr;
  double num = 0.0, den = 0.0;
  for (int j = lane; j < nr; j += 64) {
    const double r = r0 + j;
    double w = (j == 0 ? 0.5 * r0 : 0.5) + (j < nr - 1 ? 0.5 : 0.0);
    if (!area) w *= (double)u[j];
    num += w * r * (double)t[j];
    den += w * r;
  }
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_xor(num, off, 64);
    den += __shfl_xor(den, off, 64);
  }
  if (lane == 0) {
    const double b = num / den;
    const double tw = t[nr - 1];
    const double g = (3.0 * tw - 4.0 * (double)t[nr - 2] + (double)t[nr - 3]) * 0.5;
    tb[k] = b;
    nu[k] = 2.0 * (r0 + (nr - 1)) * g / (tw - b);
  }
}

// out[0] = max of colmax[0..n) (one block).
__global__ __launch_bounds__(RB) void k_absmax(const double* __restrict__ colmax, int n,
                                               double* __restrict__ out) {
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += RB) mx = fmax(mx, colmax[i]);
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  __shared__ double sh[RB / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < RB / 64; ++i) mx = fmax(mx, sh[i]);
    out[0] = fmax(mx, sh[0]);
  }
}

// ---- host side ------------------------------------------------------------------

namespace {

int validate(const lbm_axi_params& p, int i) {
  const std::string pre = "instance " + std::to_string(i) + ": ";
  if (p.side_rmin < 0 || p.side_rmin > 2 || p.side_rmax < 0 || p.side_rmax > 2 || p.side_z < 0 ||
      p.side_z > 3)
    return fail(LBM_AXI_EINVAL, pre + "side code out of range (inlet/outlet along z only)");
  if (p.side_z == SIDE_AXIS) return fail(LBM_AXI_EINVAL, pre + "the z sides cannot be an axis");
  if (p.side_rmax == SIDE_AXIS) return fail(LBM_AXI_EINVAL, pre + "the axis can only be at r_min");
  if ((p.side_rmin == SIDE_PERIODIC) != (p.side_rmax == SIDE_PERIODIC))
    return fail(LBM_AXI_EINVAL, pre + "radial periodicity needs both r sides periodic");
  if (p.side_rmin == SIDE_AXIS && p.r0 != 0.5)
    return fail(LBM_AXI_EINVAL, pre + "an axis needs r0 = 1/2 (cell-centred rows)");
  if (p.nr < 3 || p.nz < 1 || ((p.side_z == SIDE_WALL || p.side_z == SIDE_FLOW) && p.nz < 3))
    return fail(LBM_AXI_EINVAL, pre + "grid too small (nr >= 3, nz >= 3 with axial boundaries)");
  if (!std::isfinite(p.u_in)) return fail(LBM_AXI_EINVAL, pre + "u_in must be finite");
  if (!(p.tail_tol >= 0.0)) return fail(LBM_AXI_EINVAL, pre + "tail_tol must be 0 or positive");
  if ((int64_t)p.nr * p.nz > (int64_t)1 << 31)
    return fail(LBM_AXI_EINVAL, pre + "grid larger than 2^31 nodes");
  if (!(p.r0 > 0.0)) return fail(LBM_AXI_EINVAL, pre + "r0 must be positive");
  if (!(p.phi > 0.0 && p.phi <= 1.0)) return fail(LBM_AXI_EINVAL, pre + "phi must lie in (0, 1]");
  if (!(p.Da > 0.0) || !(p.L > 0.0)) return fail(LBM_AXI_EINVAL, pre + "Da and L must be positive");
  if (!(p.J > 0.0) || !(p.Pr > 0.0) || !(p.lambda > 0.0))
    return fail(LBM_AXI_EINVAL, pre + "J, Pr and lambda must be positive");
  if (p.sigma != 1.0)
    return fail(LBM_AXI_EUNSUPPORTED, pre + "only a heat-capacity ratio of 1 is defined (Eq. 4)");
  if (p.storage < 0 || p.storage > 2) return fail(LBM_AXI_EINVAL, pre + "storage code out of range");
  if (p.therm_rmin < 0 || p.therm_rmin > 2 || p.therm_rmax < 0 || p.therm_rmax > 2 || p.therm_z < 0 ||
      p.therm_z > 1)
    return fail(LBM_AXI_EINVAL, pre + "thermal code out of range (flux walls are radial only)");
  if (!std::isfinite(p.flux_rmin) || !std::isfinite(p.flux_rmax) || std::isnan(p.flux_zlo) ||
      std::isnan(p.flux_zhi))
    return fail(LBM_AXI_EINVAL, pre + "flux values must be finite and the window not NaN");
  if (p.check_interval == 1 || p.check_interval < 0)
    return fail(LBM_AXI_EINVAL, pre + "check_interval must be 0 or >= 2");
  if (!(p.tau_nu > 0.0) && !(p.Ra > 0.0))
    return fail(LBM_AXI_EINVAL, pre + "give tau_nu or a positive Ra (Eq. 39)");
  return LBM_AXI_OK;
}

// Default nodes per thread along z, per parity of the AA step: the largest of
// 1 (FP32 even steps), 2 (FP32 odd steps) or 8 (16-bit storage), halving down
// to 1, that still gives the launch at least 512 blocks.  Small grids are
// latency-bound: each thread's nodes run one after another, so fewer nodes
// per thread shorten the critical path (measured on 100 x 200 and 256^2:
// kz = 1 steps in 6.3 us against 15 us at kz = 4); large grids are
// bandwidth-bound, and at 8192^2 the FP32 even step is fastest at kz = 1
// (1.41 ms; 1.46 at kz = 2), the odd step at kz = 2 (1.55 ms; 1.87 at
// kz = 1), both 16-bit steps at kz = 8 (0.95 / 0.98 ms).
int default_kz(const lbm_axi* h, bool odd = false) {
  const int kmax = h->storage == LBM_STORE_FP32 ? (odd ? 2 : 1) : 8;
  for (int kz = kmax; kz > 1; kz /= 2) {
    long long blocks = 0;
    for (const lbm_axi_params& q : h->prm)
      blocks += (long long)((q.nr + BX - 1) / BX) * ((q.nz + BY * kz - 1) / (BY * kz));
    if (blocks >= 512) return kz;
  }
  return 1;
}

// Share of the step's waves (column groups of BX lanes, weighted by nz) that
// hold a radial wall lane, over every instance of the handle.  Without wall
// lanes such a wave runs its owner's wall node after the owner's update
// (measured: about 2.1 times an interior wave); with them the wall lanes run
// a short tail of their own (about 1.5 times), but every wave of the kernel
// carries about 20 more VGPRs (FP32 even steps drop from 4 to 3 waves per
// SIMD, 3 % slower at 8192^2).  Wall lanes therefore pay above a few per
// cent: measured 1.20 against 1.44 ms per step for the 1024-instance sweep
// (42 % of waves), 0.935 against 0.922 ms at 8192^2 in FP16 (1.6 %).  The
// choice depends on the instances only, so compaction and launch shapes keep
// results bit-identical.
double wall_wave_share(const lbm_axi* h) {
  double all = 0.0, wall = 0.0;
  for (const InstDev& D : h->hdesc) {
    const int ncol = (D.nr + BX - 1) / BX;
    const bool lo = D.side_rmin == SIDE_WALL;
    const bool hi = D.side_rmax == SIDE_WALL && wall_lane_rmax(D);
    const int walls = (lo ? 1 : 0) + (hi && !(lo && (D.nr - 1) / BX == 0) ? 1 : 0);
    all += (double)ncol * D.nz;
    wall += (double)walls * D.nz;
  }
  return all > 0.0 ? wall / all : 0.0;
}
bool default_wall_lanes(const lbm_axi* h) { return wall_wave_share(h) > 0.05; }

// Byte size for buffer addressing (32-bit offsets), 0 when 4 GiB or more.
uint32_t pop_bytes32(size_t bytes) { return bytes < 0xFFFFFFFFull ? (uint32_t)bytes : 0u; }

bool all_buffer_addressable(const lbm_axi* h) {
  for (const InstDev& D : h->hdesc)
    if (D.pop_bytes == 0) return false;
  return !h->hdesc.empty() && h->storage != LBM_STORE_FP32;
}

void* dalloc(lbm_axi* h, size_t bytes, hipError_t* err) {
  void* p = nullptr;
  *err = hipMalloc(&p, bytes);
  if (*err != hipSuccess) return nullptr;
  h->allocs.push_back(p);
  h->bytes += bytes;
  return p;
}

// Launch description of the step over the handle's tile list of one parity
// (on stream st), and over one instance's plain tile list.
StepLaunch step_launch(const lbm_axi* h, bool odd, hipStream_t st) {
  return StepLaunch{h->ddesc, odd ? h->dtiles_odd : h->dtiles, h->dstatus,
                    odd ? h->ntiles_odd : h->ntiles_launch, odd ? h->kz_odd : h->kz, h->lds_bytes, st};
}
StepLaunch inst_launch(const lbm_axi* h, int inst) {
  return StepLaunch{h->ddesc, h->dtiles_plain + h->tile_first[inst], h->dstatus, h->tile_count[inst],
                    h->kz, 0, h->stream};
}

int launch_result(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(LBM_AXI_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return LBM_AXI_OK;
}

// One step launch in the handle's storage type.  16-bit storage takes buffer
// addressing when buf (every instance's population array below 4 GiB;
// measured 12 % faster at 8192^2); FP32 keeps flat addressing: there the
// buffer form, though lighter on registers, measured 15 % slower.
int launch_step(lbm_axi* h, bool buf, bool odd, int mode, const StepLaunch& L, int slot, uint32_t seed,
                const long long* clk, int off) {
  hipError_t e;
  if (h->storage == LBM_STORE_FP32)
    e = launch_step_b<float, false>(h->wall_lanes, odd, mode, L, slot, seed, clk, off);
  else
    e = launch_step_s16(h->storage, buf, h->wall_lanes, odd, mode, L, slot, seed, clk, off);
  return launch_result(e, "step kernel launch");
}

int launch_fields(lbm_axi* h, int inst, bool odd, const FieldOut& fo) {
  const StepLaunch L = inst_launch(h, inst);
  return launch_result(h->storage == LBM_STORE_FP32 ? launch_fields_t<float>(odd, L, fo)
                                                    : launch_fields_s16(h->storage, odd, L, fo),
                       "field kernel launch");
}

// The probe takes the step's addressing: buffer addressing for 16-bit
// storage when every array is below 4 GiB, flat otherwise.
int launch_pattern(lbm_axi* h, bool odd, uint32_t key) {
  const StepLaunch L = step_launch(h, odd, h->stream);
  return launch_result(h->storage == LBM_STORE_FP32 ? launch_pattern_t<float, false>(odd, L, key)
                                                    : launch_pattern_s16(h->storage, h->buf, odd, L, key),
                       "pattern kernel launch");
}

int launch_init(lbm_axi* h, int inst, const float* dinit, float T_init) {
  const StepLaunch L = inst_launch(h, inst);
  return launch_result(h->storage == LBM_STORE_FP32 ? launch_init_t<float>(L, dinit, T_init, inst)
                                                    : launch_init_s16(h->storage, L, dinit, T_init, inst),
                       "start kernel launch");
}

// Tiles of BX lanes along r by BY * kz rows along z, for every instance.
// Launch order: block b takes tile (b % 8) * ceil(T / 8) + b / 8, so that
// the 8 XCDs, which receive blocks round-robin, each sweep a contiguous run
// of tiles (neighbouring rows share that XCD's L2).
// Only instances flagged in h->active (all when it is empty) enter the launch
// list; the per-instance list (field output) always holds every instance.
int build_tiles(lbm_axi* h, int kz, int kz_odd) {
  // Per-instance list in instance order (field and start kernels, strips of kz)
  // and, for each parity, the XCD-ordered list of the running instances.
  std::vector<int4> tiles;
  std::vector<int> first, count;
  for (int i = 0; i < h->n_inst; ++i) {
    const lbm_axi_params& q = h->prm[i];
    first.push_back((int)tiles.size());
    for (int k0 = 0; k0 < q.nz; k0 += BY * kz)
      for (int j0 = 0; j0 < q.nr; j0 += BX) tiles.push_back(make_int4(i, j0, k0, 0));
    count.push_back((int)tiles.size() - first.back());
  }
  auto ordered = [&](int kzp) {
    std::vector<int4> live;
    for (int i = 0; i < h->n_inst; ++i) {
      if (!(h->active.empty() || h->active[i])) continue;
      const lbm_axi_params& q = h->prm[i];
      // A row's last column tile, when at most half a wave wide, is packed:
      // one tile (w = 1) takes two consecutive z strips, one per half wave.
      // Half-empty waves cost nearly a full wave at 2-byte lanes (measured:
      // the 1024-instance sweep, 5.7 % of its waves).
      for (int k0 = 0, s = 0; k0 < q.nz; k0 += BY * kzp, ++s)
        for (int j0 = 0; j0 < q.nr; j0 += BX) {
          if (q.nr - j0 <= BX / 2) {
            if (s % 2 == 0) live.push_back(make_int4(i, j0, k0, 1));
          } else {
            live.push_back(make_int4(i, j0, k0, 0));
          }
        }
    }
    const int T = (int)live.size();
    const int per = T > 0 ? (T + 7) / 8 : 1;
    std::vector<int4> order((size_t)per * 8, make_int4(-1, 0, 0, 0));
    for (int b = 0; b < per * 8; ++b) {
      const int t = (b % 8) * per + b / 8;
      if (t < T) order[b] = live[t];
    }
    return order;
  };
  const std::vector<int4> even = ordered(kz), odd = ordered(kz_odd);
  int4 *dt = nullptr, *dto = nullptr, *dp = nullptr;
  auto free_new = [&]() {
    for (int4* x : {dt, dto, dp})
      if (x) (void)hipFree(x);
  };
  if (hipMalloc(&dt, sizeof(int4) * even.size()) != hipSuccess ||
      hipMalloc(&dto, sizeof(int4) * odd.size()) != hipSuccess ||
      hipMalloc(&dp, sizeof(int4) * tiles.size()) != hipSuccess) {
    free_new();
    return fail(LBM_AXI_ENOMEM, "tile lists");
  }
  if (hipMemcpy(dt, even.data(), sizeof(int4) * even.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dto, odd.data(), sizeof(int4) * odd.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dp, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess) {
    free_new();
    return fail(LBM_AXI_EDEVICE, "tile list upload");
  }
  if (h->dtiles) (void)hipFree(h->dtiles);
  if (h->dtiles_odd) (void)hipFree(h->dtiles_odd);
  if (h->dtiles_plain) (void)hipFree(h->dtiles_plain);
  h->dtiles = dt;
  h->dtiles_odd = dto;
  h->dtiles_plain = dp;
  h->ntiles_launch = (int)even.size();
  h->ntiles_odd = (int)odd.size();
  h->tile_first = first;
  h->tile_count = count;
  h->kz = kz;
  h->kz_odd = kz_odd;
  return LBM_AXI_OK;
}

int dispatch_step(lbm_axi* h, bool odd, int mode, int slot, uint32_t seed,
                  hipStream_t st = nullptr, const long long* clk = nullptr, int off = 0) {
  if (!st) st = h->stream;
  return launch_step(h, h->buf, odd, mode, step_launch(h, odd, st), slot, seed, clk, off);
}

void drop_graph(lbm_axi* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
}

// Captures graph_steps plain steps starting at an even time level (parity
// even, odd, even, ...), each reading its time level from the device clock.
int capture_graph(lbm_axi* h) {
  drop_graph(h);
  if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(LBM_AXI_EDEVICE, "capture stream");
  HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = LBM_AXI_OK;
  for (int i = 0; i < h->graph_steps && rc == LBM_AXI_OK; ++i)
    rc = dispatch_step(h, (i & 1) != 0, MODE_STEP, 0, 0u, h->cap_stream, h->dclk, i);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess || !g) return fail(LBM_AXI_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  h->graph = g;
  if (hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
    drop_graph(h);
    return fail(LBM_AXI_EDEVICE, "graph instantiation");
  }
  return LBM_AXI_OK;
}

template <typename Si, typename So>
void launch_convert(lbm_axi* h, const InstDev& Di, const InstDev& Do) {
  const int64_t nb = (Di.plane + RB - 1) / RB;
  k_convert<Si, So><<<(unsigned)nb, RB, 0, h->stream>>>(Di, Do);
}

template <typename Si>
void launch_convert_to(lbm_axi* h, int to, const InstDev& Di, const InstDev& Do) {
  switch (to) {
    case LBM_STORE_FP32: launch_convert<Si, float>(h, Di, Do); break;
    case LBM_STORE_FP16: launch_convert<Si, __half>(h, Di, Do); break;
    default: launch_convert<Si, __hip_bfloat16>(h, Di, Do); break;
  }
}

void release(lbm_axi* h, void* p, size_t bytes) {
  for (size_t i = 0; i < h->allocs.size(); ++i)
    if (h->allocs[i] == p) {
      h->allocs.erase(h->allocs.begin() + (long)i);
      (void)hipFree(p);
      h->bytes -= bytes;
      return;
    }
}

// One step of instance inst alone, in the AA layout of parity `odd` (plain
// tile list, flat addressing, the handle's wall-lane variant).
int launch_inst_step(lbm_axi* h, int inst, bool odd, uint32_t seed) {
  return launch_step(h, false, odd, MODE_STEP, inst_launch(h, inst), 0, seed, nullptr, 0);
}

// Sets converged instances running again (after a storage conversion).  A
// stopped instance's populations sit at the handle level t_stop at which it
// stopped, in that level's AA layout, while the handle has moved on to h->t.
// If the two levels differ in parity the instance first takes one step on its
// own, so that its layout is the one the handle's next step expects.  The
// handle steps it sat out are added to t_off (an even number), so that its
// own time level stays continuous, and its first check after the restart only
// records (its other check buffer is stale).  Stalled and diverged instances
// stay stopped.
int resume_converged(lbm_axi* h) {
  const int n = h->n_inst;
  std::vector<int> st(n);
  std::vector<DevResult> rr(n);
  HIPCHK(hipMemcpy(st.data(), h->dstatus, sizeof(int) * n, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(rr.data(), h->dres, sizeof(DevResult) * n, hipMemcpyDeviceToHost));
  std::vector<int> resumed;
  for (int i = 0; i < n; ++i)
    if (st[i] == CONVERGED && rr[i].t_stop >= 0 && rr[i].t_stop <= h->t) {
      st[i] = RUN;
      resumed.push_back(i);
    }
  if (resumed.empty()) return LBM_AXI_OK;
  HIPCHK(hipMemcpy(h->dstatus, st.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  const long long N = h->check > 0 ? h->check : 1;
  for (int i : resumed) {
    DevResult& r = rr[i];
    const long long gap = h->t - r.t_stop;
    if (gap & 1) {
      const bool odd = (r.t_stop & 1) != 0;
      const uint32_t seed = step_seed(r.t_stop - r.t_off);
      const int rc = launch_inst_step(h, i, odd, seed);
      if (rc) return rc;
    }
    r.t_off += gap - (gap & 1);
    r.t_arm = (h->t + N - 1) / N * N + N;
    r.t_stop = -1;
    r.res = r.res_u = r.res_T = r.ru_prev = r.rT_prev = HUGE_VAL;
    r.dnu_i_prev = r.dnu_o_prev = HUGE_VAL;
  }
  HIPCHK(hipMemcpyAsync(h->dres, rr.data(), sizeof(DevResult) * n, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (!h->active.empty()) {
    for (int i : resumed) h->active[i] = 1;
    drop_graph(h);
    return build_tiles(h, h->kz, h->kz_odd);
  }
  return LBM_AXI_OK;
}

// Host-side failures (allocation) become error codes: nothing may unwind
// through the C ABI.
template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(LBM_AXI_ENOMEM, "host memory exhausted");
  } catch (const std::exception& e) {
    return fail(LBM_AXI_EDEVICE, e.what());
  }
}

}  // namespace

extern "C" {

void lbm_axi_default_params(lbm_axi_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->side_rmin = p->side_rmax = p->side_z = LBM_SIDE_WALL;
  p->therm_rmin = p->therm_rmax = LBM_T_FIXED;
  p->therm_z = LBM_T_ADIABATIC;
  p->flux_zlo = -HUGE_VAL;
  p->flux_zhi = HUGE_VAL;
  p->storage = LBM_STORE_FP32;
  p->storage_shift = 0;
  p->check_interval = 100;
  p->r0 = 1.0;
  p->L = 1.0;
  p->phi = 1.0;
  p->Da = 1e8;
  p->J = p->lambda = p->sigma = 1.0;
  p->Pr = 1.0;
  p->Ma = 0.1;
  p->s_e = p->s_eps = 1.1;
  p->s_q = 1.2;
  p->s_j = 1.0;
}

const char* lbm_axi_last_error(void) { return g_err.c_str(); }

void lbm_axi_destroy(lbm_axi* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (auto& e : h->ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  drop_graph(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->dtiles) (void)hipFree(h->dtiles);
  if (h->dtiles_odd) (void)hipFree(h->dtiles_odd);
  if (h->dtiles_plain) (void)hipFree(h->dtiles_plain);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

int lbm_axi_create(const lbm_axi_params* p, int32_t n_inst, const float* const* phi_field,
                   const float* const* init_uzurT, void* hip_stream, lbm_axi** out) {
  return guarded([&]() -> int {
    if (out) *out = nullptr;
    if (!p || !out || n_inst < 1) return fail(LBM_AXI_EINVAL, "null argument or n_inst < 1");
    for (int i = 0; i < n_inst; ++i) {
      int rc = validate(p[i], i);
      if (rc) return rc;
      if (p[i].storage != p[0].storage)
        return fail(LBM_AXI_EINVAL, "all instances must use the same storage");
      if (p[i].check_interval != p[0].check_interval)
        return fail(LBM_AXI_EINVAL, "all instances must use the same check_interval");
      if (phi_field && phi_field[i]) {
        if (!(p[i].phi > 0.0 && p[i].phi < 1.0))
          return fail(LBM_AXI_EINVAL, "a porosity field needs a reference porosity in (0, 1)");
        const int64_t n = (int64_t)p[i].nr * p[i].nz;
        for (int64_t c = 0; c < n; ++c)
          if (!(phi_field[i][c] > 0.0f && phi_field[i][c] < 1.0f))
            return fail(LBM_AXI_EINVAL, "porosity field values must lie in (0, 1)");
      }
    }
    lbm_axi* h = new lbm_axi();
    h->n_inst = n_inst;
    h->storage = p[0].storage;
    h->check = p[0].check_interval;
    h->prm.assign(p, p + n_inst);
    h->kz = default_kz(h);  // needs the problem sizes
    h->kz_odd = default_kz(h, true);
    auto bail = [&](int rc) {
      lbm_axi_destroy(h);
      return rc;
    };
  #define HIPBAIL(call)                                                                       \
    do {                                                                                      \
      hipError_t e_ = (call);                                                                 \
      if (e_ != hipSuccess)                                                                   \
        return bail(fail(LBM_AXI_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_))); \
    } while (0)
    {
      int dev = 0, lds = 0, ldsb = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
          hipDeviceGetAttribute(&ldsb, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return bail(fail(LBM_AXI_EDEVICE, "device query failed"));
      h->lds_per_cu = lds;
      h->lds_per_block = ldsb;
      h->device = dev;
      // Device address of the static scratch array, resolved once per device
      // with that device current (it is the current one here).
      if (dev < 0 || dev >= MAX_DEVICES) return bail(fail(LBM_AXI_EDEVICE, "device index out of range"));
      std::lock_guard<std::mutex> lock(g_scratch_mu);
      if (!g_scratch[dev]) {
        void* sp = nullptr;
        const hipError_t se = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
        if (se != hipSuccess || !sp)
          return bail(fail(LBM_AXI_EDEVICE, std::string("scratch address: ") + hipGetErrorString(se)));
        g_scratch[dev] = sp;
      }
      h->scratch = g_scratch[dev];
    }
    if (hip_stream) {
      h->stream = (hipStream_t)hip_stream;
    } else {
      if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(LBM_AXI_EDEVICE, "hipStreamCreate failed"));
      h->own_stream = true;
    }
    const size_t esz = h->storage == LBM_STORE_FP32 ? 4 : 2;
    hipError_t err = hipSuccess;
    h->hdesc.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
      const lbm_axi_params& q = p[i];
      InstDev& D = h->hdesc[i];
      const bool field = phi_field && phi_field[i];
      {
        std::string msg;
        const int rc = describe(q, field, D, msg);
        if (rc) return bail(fail(rc, msg));
      }
      D.pop = dalloc(h, (size_t)14 * D.plane * esz, &err);
      D.pop_bytes = pop_bytes32((size_t)14 * D.plane * esz);
      if (!D.pop) return bail(fail(LBM_AXI_ENOMEM, std::string("population array: ") + hipGetErrorString(err)));
      if (h->storage == LBM_STORE_FP32) {
        D.g0 = (float*)D.pop + 9 * D.plane;
      } else {
        D.g0 = (float*)dalloc(h, (size_t)D.plane * 4, &err);
        if (!D.g0) return bail(fail(LBM_AXI_ENOMEM, std::string("g_0 plane: ") + hipGetErrorString(err)));
      }
      if (field) {
        float* dphi = (float*)dalloc(h, (size_t)D.plane * 4, &err);
        if (!dphi) return bail(fail(LBM_AXI_ENOMEM, "porosity field"));
        std::vector<float> pad((size_t)D.plane, q.phi);
        for (int k = 0; k < q.nz; ++k)
          std::memcpy(&pad[(size_t)k * D.stride], phi_field[i] + (size_t)k * q.nr, sizeof(float) * q.nr);
        if (hipMemcpy(dphi, pad.data(), sizeof(float) * D.plane, hipMemcpyHostToDevice) != hipSuccess)
          return bail(fail(LBM_AXI_EDEVICE, "porosity field upload"));
        D.phi = dphi;
      }
      if (h->check > 0) {
        for (int s = 0; s < 2; ++s) {
          D.mac[s] = (float*)dalloc(h, (size_t)3 * D.plane * 4, &err);
          if (!D.mac[s]) return bail(fail(LBM_AXI_ENOMEM, "check buffers"));
          if (hipMemset(D.mac[s], 0, (size_t)3 * D.plane * 4) != hipSuccess)
            return bail(fail(LBM_AXI_EDEVICE, "check buffer clear"));
        }
      }
    }
    {
      const int rc = build_tiles(h, h->kz, h->kz_odd);
      if (rc) return bail(rc);
    }
    h->ddesc = (InstDev*)dalloc(h, sizeof(InstDev) * n_inst, &err);
    h->dstatus = (int*)dalloc(h, sizeof(int) * n_inst, &err);
    h->dclk = (long long*)dalloc(h, sizeof(long long), &err);
    h->dres = (DevResult*)dalloc(h, sizeof(DevResult) * n_inst, &err);
    if (!h->ddesc || !h->dstatus || !h->dres || !h->dclk)
      return bail(fail(LBM_AXI_ENOMEM, "descriptor arrays"));
    HIPBAIL(hipMemcpy(h->ddesc, h->hdesc.data(), sizeof(InstDev) * n_inst, hipMemcpyHostToDevice));
    h->buf = all_buffer_addressable(h);
    h->wall_lanes = default_wall_lanes(h);
    HIPBAIL(hipMemset(h->dstatus, 0, sizeof(int) * n_inst));
    {
      std::vector<DevResult> r0(n_inst);
      for (auto& r : r0) {
        r.res = r.res_u = r.res_T = HUGE_VAL;
        r.nu_i = r.nu_o = r.u_rms = 0.0;
        r.t_check = -1;
        r.t_stop = -1;
        r.t_off = 0;
        r.t_arm = h->check;  // the check at level 0 only fills a buffer
        r.ru_prev = r.rT_prev = r.dnu_i_prev = r.dnu_o_prev = HUGE_VAL;
        r.nu_i_prev = r.nu_o_prev = 0.0;
      }
      HIPBAIL(hipMemcpy(h->dres, r0.data(), sizeof(DevResult) * n_inst, hipMemcpyHostToDevice));
    }
    // Reduction tiles: RZ rows per block.
    if (h->check > 0) {
      std::vector<ResTile> rts;
      std::vector<int> first(2 * n_inst);
      std::vector<double> tol(n_inst), tail(n_inst), nus(4 * n_inst);
      std::vector<long long> mx(n_inst);
      for (int i = 0; i < n_inst; ++i) {
        const int nz = p[i].nz, nr = p[i].nr;
        int rz = std::max(1, (int)((8192 + nr - 1) / nr));  // about 8k nodes per block
        first[2 * i] = (int)rts.size();
        for (int k0 = 0; k0 < nz; k0 += rz) rts.push_back(ResTile{i, k0, std::min(nz, k0 + rz), 0});
        first[2 * i + 1] = (int)rts.size() - first[2 * i];
        tol[i] = p[i].tol;
        tail[i] = p[i].tail_tol;
        mx[i] = p[i].max_steps;
        const double dT = p[i].delta_T != 0.0 ? p[i].delta_T : p[i].T_rmin - p[i].T_rmax;
        const double H = nz - 1;
        const bool walls = p[i].side_rmin == SIDE_WALL && p[i].side_rmax == SIDE_WALL && dT != 0.0 && H > 0;
        nus[4 * i] = walls ? p[i].r0 / (H * dT) : 0.0;
        nus[4 * i + 1] = (p[i].side_rmax == SIDE_WALL && dT != 0.0 && H > 0)
                             ? (p[i].r0 + nr - 1) / (H * dT) : 0.0;
        // Isoflux walls: Nu = (q'/k) L / n_heated * sum 1 / (T_h - T_0) (NaN if unheated).
        for (int side = 0; side < 2; ++side) {
          if ((side ? p[i].therm_rmax : p[i].therm_rmin) != LBM_T_FLUX) continue;
          const InstDev& D = h->hdesc[i];
          const int j = side ? nr - 1 : 0;
          int cnt = 0;
          float qf;
          for (int k = 0; k < nz; ++k)
            if (is_boundary(D, j, k) && flux_node(D, node_mask(D, j, k), k, qf)) ++cnt;
          const double qv = side ? p[i].flux_rmax : p[i].flux_rmin;
          nus[4 * i + side] = cnt ? -qv * p[i].L / cnt : NAN;
        }
        // residual scales: 1 / (Ma c_s) and 1 / |dT|
        nus[4 * i + 2] = p[i].Ma > 0.0 ? 1.0 / (p[i].Ma * std::sqrt(1.0 / 3.0)) : 1.0;
        nus[4 * i + 3] = dT != 0.0 ? 1.0 / std::fabs(dT) : 1.0;
      }
      h->nrt = (int)rts.size();
      h->drt = (ResTile*)dalloc(h, sizeof(ResTile) * rts.size(), &err);
      h->dpart = (double*)dalloc(h, sizeof(double) * 6 * rts.size(), &err);
      h->dfirst = (int*)dalloc(h, sizeof(int) * first.size(), &err);
      h->dtol = (double*)dalloc(h, sizeof(double) * n_inst, &err);
      h->dtail = (double*)dalloc(h, sizeof(double) * n_inst, &err);
      h->dnus = (double*)dalloc(h, sizeof(double) * 4 * n_inst, &err);
      h->dmx = (long long*)dalloc(h, sizeof(long long) * n_inst, &err);
      if (!h->drt || !h->dpart || !h->dfirst || !h->dtol || !h->dtail || !h->dnus || !h->dmx)
        return bail(fail(LBM_AXI_ENOMEM, "reduction arrays"));
      HIPBAIL(hipMemcpy(h->drt, rts.data(), sizeof(ResTile) * rts.size(), hipMemcpyHostToDevice));
      HIPBAIL(hipMemcpy(h->dfirst, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice));
      HIPBAIL(hipMemcpy(h->dtol, tol.data(), sizeof(double) * n_inst, hipMemcpyHostToDevice));
      HIPBAIL(hipMemcpy(h->dtail, tail.data(), sizeof(double) * n_inst, hipMemcpyHostToDevice));
      HIPBAIL(hipMemcpy(h->dnus, nus.data(), sizeof(double) * 4 * n_inst, hipMemcpyHostToDevice));
      HIPBAIL(hipMemcpy(h->dmx, mx.data(), sizeof(long long) * n_inst, hipMemcpyHostToDevice));
    }
    // Start state of every instance.
    for (int i = 0; i < n_inst; ++i) {
      float* dinit = nullptr;
      if (init_uzurT && init_uzurT[i]) {
        const size_t n = (size_t)p[i].nr * p[i].nz;
        if (hipMalloc(&dinit, sizeof(float) * 3 * n) != hipSuccess)
          return bail(fail(LBM_AXI_ENOMEM, "start-field staging"));
        if (hipMemcpy(dinit, init_uzurT[i], sizeof(float) * 3 * n, hipMemcpyHostToDevice) != hipSuccess) {
          (void)hipFree(dinit);
          return bail(fail(LBM_AXI_EDEVICE, "start-field upload"));
        }
      }
      int rc;
      rc = launch_init(h, i, dinit, (float)p[i].T_init);
      if (dinit) {
        hipError_t e = hipStreamSynchronize(h->stream);
        (void)hipFree(dinit);
        if (e != hipSuccess) return bail(fail(LBM_AXI_EDEVICE, std::string("start state: ") + hipGetErrorString(e)));
      }
      if (rc) return bail(rc);
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess)
      return bail(fail(LBM_AXI_EDEVICE, "start state"));
    *out = h;
    return LBM_AXI_OK;
  #undef HIPBAIL
  });
}

int lbm_axi_step(lbm_axi* h, int32_t nsteps) {
  return guarded([&]() -> int {
    if (!h || nsteps < 0) return fail(LBM_AXI_EINVAL, "null handle or negative step count");
    const long long t_end = h->t + nsteps;
    while (h->t < t_end) {
      const long long n = h->t;
      // A run of graph_steps plain steps from an even level with no check step
      // inside goes through the captured graph (not while timing launches).
      const int G = h->graph_steps;
      if (G >= 2 && !h->timing && (n & 1) == 0 && n + G <= t_end &&
          (h->check <= 0 || (n + h->check - 1) / h->check * h->check >= n + G)) {
        if (!h->gexec) {
          const int rc = capture_graph(h);
          if (rc) return rc;
        }
        k_setclock<<<1, 1, 0, h->stream>>>(h->dclk, n);
        HIPCHK(hipGetLastError());
        HIPCHK(hipGraphLaunch(h->gexec, h->stream));
        h->t = n + G;
        continue;
      }
      const bool odd = (n & 1) != 0;
      // At every multiple of the check interval the step also writes u_z, u_r,
      // T into one of two buffers (alternating); from the second one on, the
      // check compares them with the previous multiple's.
      int mode = MODE_STEP, slot = 0;
      bool check = false;
      if (h->check > 0 && n % h->check == 0) {
        mode = MODE_STEP_MACRO;
        slot = (int)((n / h->check) & 1);
        check = n > 0;
      }
      if (h->timing) {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        h->ev.emplace_back(e0, e1);
        HIPCHK(hipEventRecord(e0, h->stream));
      }
      // random bits of this step for stochastic rounding (16-bit storage)
      int rc = dispatch_step(h, odd, mode, slot, step_seed(n));
      if (rc) return rc;
      if (h->timing) {
        HIPCHK(hipEventRecord(h->ev.back().second, h->stream));
        if (h->ev.size() >= 1024) {
          double ms;
          int64_t nl;
          rc = lbm_axi_kernel_time(h, &ms, &nl);
          if (rc) return rc;
        }
      }
      if (check) {
        k_resid<<<h->nrt, RB, 0, h->stream>>>(h->ddesc, h->drt, slot, h->dstatus, h->dpart);
        HIPCHK(hipGetLastError());
        k_final<<<h->n_inst, RB, 0, h->stream>>>(h->dfirst, h->dpart, n, 1.0 / h->check, h->dtol,
                                                  h->dtail, h->dmx, h->dnus, h->dstatus, h->dres);
        HIPCHK(hipGetLastError());
      }
      h->t = n + 1;
    }
    return LBM_AXI_OK;
  });
}

int lbm_axi_set_graph(lbm_axi* h, int32_t steps) {
  return guarded([&]() -> int {
    if (!h || steps < 0 || steps > 4096 || (steps & 1))
      return fail(LBM_AXI_EINVAL, "bad handle or graph steps not an even number in [0, 4096]");
    HIPCHK(hipStreamSynchronize(h->stream));
    drop_graph(h);
    h->graph_steps = steps;
    return LBM_AXI_OK;
  });
}

int lbm_axi_compact(lbm_axi* h, int32_t* n_running) {
  return guarded([&]() -> int {
    if (!h) return fail(LBM_AXI_EINVAL, "null handle");
    std::vector<int> st(h->n_inst);
    HIPCHK(hipMemcpyAsync(st.data(), h->dstatus, sizeof(int) * h->n_inst, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    std::vector<char> act(h->n_inst);
    int nr = 0;
    for (int i = 0; i < h->n_inst; ++i) {
      act[i] = st[i] == RUN;
      nr += act[i];
    }
    if (n_running) *n_running = nr;
    if (act == h->active || (h->active.empty() && nr == h->n_inst)) return LBM_AXI_OK;
    h->active = act;
    drop_graph(h);
    return build_tiles(h, h->kz, h->kz_odd);
  });
}

int lbm_axi_autotune(lbm_axi* h, int32_t trial_steps, int32_t* kz_out, int32_t* bpc_out,
                     double* ms_out) {
  return guarded([&]() -> int {
    if (!h || trial_steps < 1) return fail(LBM_AXI_EINVAL, "null handle or trial_steps < 1");
    static const int KZ[] = {1, 2, 4, 8, 16};
    static const int BPC[] = {0, 2, 4};
    const bool was_timing = h->timing;
    double best = HUGE_VAL;
    int bk = h->kz, bb = 0;
    for (int kz : KZ)
      for (int bpc : BPC) {
        int rc = lbm_axi_set_tiles(h, kz, bpc);
        if (rc) return rc;
        h->timing = false;
        rc = lbm_axi_set_timing(h, 1);  // restarts the launch timer
        if (rc) return rc;
        rc = lbm_axi_step(h, trial_steps);
        if (rc) return rc;
        double ms = 0.0;
        int64_t nl = 0;
        rc = lbm_axi_kernel_time(h, &ms, &nl);
        if (rc) return rc;
        const double per = nl > 0 ? ms / (double)nl : HUGE_VAL;
        if (per < best) {
          best = per;
          bk = kz;
          bb = bpc;
        }
      }
    h->timing = false;
    int rc = lbm_axi_set_timing(h, was_timing ? 1 : 0);
    if (rc) return rc;
    rc = lbm_axi_set_tiles(h, bk, bb);
    if (rc) return rc;
    if (kz_out) *kz_out = bk;
    if (bpc_out) *bpc_out = bb;
    if (ms_out) *ms_out = best;
    return LBM_AXI_OK;
  });
}

int lbm_axi_set_storage(lbm_axi* h, int32_t storage, int32_t storage_shift) {
  return guarded([&]() -> int {
    if (!h || storage < LBM_STORE_FP32 || storage > LBM_STORE_BF16 || storage_shift < 0 ||
        storage_shift > 24)
      return fail(LBM_AXI_EINVAL, "bad handle, storage type or storage_shift out of [0, 24]");
    HIPCHK(hipStreamSynchronize(h->stream));
    drop_graph(h);
    const int from = h->storage;
    const size_t esz_o = from == LBM_STORE_FP32 ? 4 : 2;
    const size_t esz_n = storage == LBM_STORE_FP32 ? 4 : 2;
    std::vector<InstDev> nd(h->n_inst);
    std::vector<lbm_axi_params> np(h->prm);
    hipError_t err = hipSuccess;
    // Allocate everything first: on failure the handle is left as it was.
    for (int i = 0; i < h->n_inst; ++i) {
      np[i].storage = storage;
      np[i].storage_shift = storage_shift;
      std::string msg;
      const InstDev& Do = h->hdesc[i];
      InstDev& Dn = nd[i];
      int rc = describe(np[i], Do.phi != nullptr, Dn, msg);
      void* pop = rc ? nullptr : dalloc(h, (size_t)14 * Dn.plane * esz_n, &err);
      float* g0 = nullptr;
      if (pop) g0 = storage == LBM_STORE_FP32 ? (float*)pop + 9 * Dn.plane
                                              : (float*)dalloc(h, (size_t)Dn.plane * 4, &err);
      if (rc || !pop || !g0) {
        for (int k = 0; k <= i; ++k) {
          if (nd[k].pop) release(h, nd[k].pop, (size_t)14 * nd[k].plane * esz_n);
          if (nd[k].g0 && storage != LBM_STORE_FP32) release(h, nd[k].g0, (size_t)nd[k].plane * 4);
        }
        if (pop) release(h, pop, (size_t)14 * Dn.plane * esz_n);
        return fail(rc ? rc : LBM_AXI_ENOMEM, rc ? msg : "population array for the new storage");
      }
      Dn.pop = pop;
      Dn.pop_bytes = pop_bytes32((size_t)14 * Dn.plane * esz_n);
      Dn.g0 = g0;
      Dn.phi = Do.phi;
      Dn.mac[0] = Do.mac[0];
      Dn.mac[1] = Do.mac[1];
    }
    hipError_t ce = hipSuccess;
    for (int i = 0; i < h->n_inst && ce == hipSuccess; ++i) {
      switch (from) {
        case LBM_STORE_FP32: launch_convert_to<float>(h, storage, h->hdesc[i], nd[i]); break;
        case LBM_STORE_FP16: launch_convert_to<__half>(h, storage, h->hdesc[i], nd[i]); break;
        default: launch_convert_to<__hip_bfloat16>(h, storage, h->hdesc[i], nd[i]); break;
      }
      ce = hipGetLastError();
    }
    if (ce == hipSuccess) ce = hipStreamSynchronize(h->stream);
    if (ce != hipSuccess) {  // keep the old state; drop the new arrays
      for (int k = 0; k < h->n_inst; ++k) {
        if (storage != LBM_STORE_FP32) release(h, nd[k].g0, (size_t)nd[k].plane * 4);
        release(h, nd[k].pop, (size_t)14 * nd[k].plane * esz_n);
      }
      return fail(LBM_AXI_EDEVICE, std::string("storage conversion: ") + hipGetErrorString(ce));
    }
    for (int i = 0; i < h->n_inst; ++i) {
      const InstDev& Do = h->hdesc[i];
      if (from != LBM_STORE_FP32) release(h, Do.g0, (size_t)Do.plane * 4);
      release(h, Do.pop, (size_t)14 * Do.plane * esz_o);
    }
    h->hdesc = nd;
    h->prm = np;
    h->storage = storage;
    h->buf = all_buffer_addressable(h);
    HIPCHK(hipMemcpy(h->ddesc, h->hdesc.data(), sizeof(InstDev) * h->n_inst, hipMemcpyHostToDevice));
    if (!h->tiles_set && (default_kz(h) != h->kz || default_kz(h, true) != h->kz_odd)) {
      const int rc = build_tiles(h, default_kz(h), default_kz(h, true));
      if (rc) return rc;
    }
    return resume_converged(h);
  });
}

int lbm_axi_set_tiles(lbm_axi* h, int32_t kz, int32_t blocks_per_cu) {
  return guarded([&]() -> int {
    if (!h || kz < 1 || kz > 64 || blocks_per_cu < 0 || blocks_per_cu > 64)
      return fail(LBM_AXI_EINVAL, "bad handle, kz out of [1, 64] or blocks_per_cu out of [0, 64]");
    HIPCHK(hipStreamSynchronize(h->stream));
    // Reserving LDS that the kernel does not use caps the blocks resident on a
    // compute unit; this is the only effect of blocks_per_cu.
    int lds = blocks_per_cu > 0 ? h->lds_per_cu / blocks_per_cu / 256 * 256 : 0;
    if (blocks_per_cu > 0 && lds * (blocks_per_cu + 1) <= h->lds_per_cu) lds += 256;
    h->lds_bytes = lds < h->lds_per_block ? lds : h->lds_per_block;
    drop_graph(h);
    h->tiles_set = true;
    return build_tiles(h, kz, kz);
  });
}

int lbm_axi_set_wall_lanes(lbm_axi* h, int32_t mode, int32_t* on) {
  return guarded([&]() -> int {
    if (!h || mode < -1 || mode > 1) return fail(LBM_AXI_EINVAL, "bad handle or mode not in {-1, 0, 1}");
    HIPCHK(hipStreamSynchronize(h->stream));
    const bool want = mode < 0 ? default_wall_lanes(h) : mode == 1;
    if (want != h->wall_lanes) drop_graph(h);  // captured graphs hold the other kernels
    h->wall_lanes = want;
    if (on) *on = want ? 1 : 0;
    return LBM_AXI_OK;
  });
}

int lbm_axi_sync(lbm_axi* h) {
  if (!h) return fail(LBM_AXI_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_AXI_OK;
}

int lbm_axi_residual(lbm_axi* h, double* res, double* nu_i, double* nu_o, int32_t* status) {
  return guarded([&]() -> int {
    if (!h) return fail(LBM_AXI_EINVAL, "null handle");
    std::vector<DevResult> r(h->n_inst);
    std::vector<int> st(h->n_inst);
    HIPCHK(hipMemcpyAsync(r.data(), h->dres, sizeof(DevResult) * h->n_inst, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(st.data(), h->dstatus, sizeof(int) * h->n_inst, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int i = 0; i < h->n_inst; ++i) {
      if (res) res[i] = r[i].res;
      if (nu_i) nu_i[i] = r[i].nu_i;
      if (nu_o) nu_o[i] = r[i].nu_o;
      if (status) status[i] = st[i];
    }
    return LBM_AXI_OK;
  });
}

int lbm_axi_info(lbm_axi* h, int32_t inst, int64_t* out) {
  if (!h || !out || inst < 0 || inst >= h->n_inst) return fail(LBM_AXI_EINVAL, "bad handle, instance or output");
  DevResult r;
  int st = 0;
  HIPCHK(hipMemcpyAsync(&r, h->dres + inst, sizeof(DevResult), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(&st, h->dstatus + inst, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  out[0] = (st == RUN ? h->t : r.t_stop) - r.t_off;
  out[1] = r.t_check;
  out[2] = st;
  out[3] = (int64_t)h->bytes;
  return LBM_AXI_OK;
}

}  // extern "C"

namespace {

// Field output of instance inst into the buffers of `out` (each may be null):
// written directly when they are device memory, else through device staging
// buffers and copied to the host (waits).
int fields_to(lbm_axi* h, int inst, const FieldOut& out, int dst_is_device) {
  return guarded([&]() -> int {
    if (!h || inst < 0 || inst >= h->n_inst) return fail(LBM_AXI_EINVAL, "bad handle or instance");
    int64_t info[4];
    int rc = lbm_axi_info(h, inst, info);
    if (rc) return rc;
    const bool odd = (info[0] & 1) != 0;
    const lbm_axi_params& q = h->prm[inst];
    const size_t n = (size_t)q.nr * q.nz;
    FieldOut fo = out;
    float *uz = out.uz, *ur = out.ur, *p = out.p, *T = out.T, *dr = out.drho;
    uint8_t* mask = out.mask;
    std::vector<void*> tmp;
    if (!dst_is_device) {
      float** fp[5] = {&fo.uz, &fo.ur, &fo.p, &fo.T, &fo.drho};
      for (float** f : fp)
        if (*f) {
          void* d = nullptr;
          if (hipMalloc(&d, sizeof(float) * n) != hipSuccess) {
            for (void* x : tmp) (void)hipFree(x);
            return fail(LBM_AXI_ENOMEM, "field staging");
          }
          tmp.push_back(d);
          *f = (float*)d;
        }
      if (fo.mask) {
        void* d = nullptr;
        if (hipMalloc(&d, n) != hipSuccess) {
          for (void* x : tmp) (void)hipFree(x);
          return fail(LBM_AXI_ENOMEM, "mask staging");
        }
        tmp.push_back(d);
        fo.mask = (uint8_t*)d;
      }
    }
    rc = launch_fields(h, inst, odd, fo);
    if (!rc && !dst_is_device) {
      hipError_t e = hipSuccess;
      if (uz && e == hipSuccess) e = hipMemcpyAsync(uz, fo.uz, sizeof(float) * n, hipMemcpyDeviceToHost, h->stream);
      if (ur && e == hipSuccess) e = hipMemcpyAsync(ur, fo.ur, sizeof(float) * n, hipMemcpyDeviceToHost, h->stream);
      if (p && e == hipSuccess) e = hipMemcpyAsync(p, fo.p, sizeof(float) * n, hipMemcpyDeviceToHost, h->stream);
      if (T && e == hipSuccess) e = hipMemcpyAsync(T, fo.T, sizeof(float) * n, hipMemcpyDeviceToHost, h->stream);
      if (mask && e == hipSuccess) e = hipMemcpyAsync(mask, fo.mask, n, hipMemcpyDeviceToHost, h->stream);
      if (dr && e == hipSuccess) e = hipMemcpyAsync(dr, fo.drho, sizeof(float) * n, hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) rc = fail(LBM_AXI_EDEVICE, std::string("field download: ") + hipGetErrorString(e));
    }
    for (void* x : tmp) (void)hipFree(x);
    return rc;
  });
}

}  // namespace

extern "C" {

int lbm_axi_macros(lbm_axi* h, int32_t inst, float* uz, float* ur, float* p, float* T,
                   uint8_t* mask, int32_t dst_is_device) {
  return fields_to(h, inst, FieldOut{uz, ur, p, T, mask, nullptr}, dst_is_device);
}

int lbm_axi_derived(const lbm_axi_params* p, double* out) {
  if (!p || !out) return fail(LBM_AXI_EINVAL, "null argument");
  const Derived d = derive(*p);
  const double v[7] = {d.tau_nu, d.tau_T, d.nu_e, d.nu, d.K_ref, d.gbeta, d.alpha_e};
  for (int i = 0; i < 7; ++i) out[i] = v[i];
  return LBM_AXI_OK;
}

int lbm_axi_density_deviation(lbm_axi* h, int32_t inst, float* drho, int32_t dst_is_device) {
  if (!drho) return fail(LBM_AXI_EINVAL, "null output");
  return fields_to(h, inst, FieldOut{nullptr, nullptr, nullptr, nullptr, nullptr, drho}, dst_is_device);
}

int lbm_axi_stream_function(lbm_axi* h, int32_t inst, float* psi, double* psi_absmax,
                            int32_t dst_is_device) {
  return guarded([&]() -> int {
    if (!h || inst < 0 || inst >= h->n_inst) return fail(LBM_AXI_EINVAL, "bad handle or instance");
    int64_t info[4];
    int rc = lbm_axi_info(h, inst, info);
    if (rc) return rc;
    const bool odd = (info[0] & 1) != 0;
    const lbm_axi_params& q = h->prm[inst];
    const size_t n = (size_t)q.nr * q.nz;
    void *duz = nullptr, *dcol = nullptr, *dmax = nullptr, *dpsi = nullptr;
    auto release_tmp = [&]() {
      (void)hipStreamSynchronize(h->stream);
      for (void* x : {duz, dcol, dmax}) (void)hipFree(x);
      if (!dst_is_device) (void)hipFree(dpsi);
    };
    bool ok = hipMalloc(&duz, sizeof(float) * n) == hipSuccess &&
              hipMalloc(&dcol, sizeof(double) * q.nz) == hipSuccess &&
              hipMalloc(&dmax, sizeof(double)) == hipSuccess;
    if (ok && psi) {
      if (dst_is_device) dpsi = psi;
      else ok = hipMalloc(&dpsi, sizeof(float) * n) == hipSuccess;
    }
    if (!ok) {
      release_tmp();
      return fail(LBM_AXI_ENOMEM, "stream function staging");
    }
    FieldOut fo{(float*)duz, nullptr, nullptr, nullptr, nullptr, nullptr};
    rc = launch_fields(h, inst, odd, fo);
    if (!rc) {
      k_psi<<<(q.nz + RB / 64 - 1) / (RB / 64), RB, 0, h->stream>>>(
          (const float*)duz, q.nr, q.nz, q.r0, q.side_rmin == LBM_SIDE_AXIS ? 1 : 0, (float*)dpsi,
          (double*)dcol);
      k_absmax<<<1, RB, 0, h->stream>>>((const double*)dcol, q.nz, (double*)dmax);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess && psi && !dst_is_device)
        e = hipMemcpyAsync(psi, dpsi, sizeof(float) * n, hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess && psi_absmax)
        e = hipMemcpyAsync(psi_absmax, dmax, sizeof(double), hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) rc = fail(LBM_AXI_EDEVICE, std::string("stream function: ") + hipGetErrorString(e));
    }
    release_tmp();
    return rc;
  });
}

int lbm_axi_stream_function_static(lbm_axi* h, int32_t inst, float* psi, double* psi_absmax) {
  return guarded([&]() -> int {
    if (!h || inst < 0 || inst >= h->n_inst) return fail(LBM_AXI_EINVAL, "bad handle or instance");
    const lbm_axi_params& q = h->prm[inst];
    if ((int64_t)q.nr * q.nz > SCRATCH_NODES || q.nz > SCRATCH_COLS)
      return fail(LBM_AXI_EINVAL, "instance larger than the static scratch (2^23 nodes, 2^16 columns)");
    if (!h->scratch) return fail(LBM_AXI_EDEVICE, "no scratch address for this device");
    int64_t info[4];
    int rc = lbm_axi_info(h, inst, info);  // run state and time level: a copy to the host, no allocation
    if (rc) return rc;
    const bool odd = (info[0] & 1) != 0;
    float* duz = (float*)h->scratch;
    double* dcol = (double*)((unsigned char*)h->scratch + SCRATCH_NODES * 4);
    FieldOut fo{duz, nullptr, nullptr, nullptr, nullptr, nullptr};
    rc = launch_fields(h, inst, odd, fo);
    if (rc) return rc;
    k_psi<<<(q.nz + RB / 64 - 1) / (RB / 64), RB, 0, h->stream>>>(
        duz, q.nr, q.nz, q.r0, q.side_rmin == LBM_SIDE_AXIS ? 1 : 0, psi, dcol);
    if (psi_absmax) k_absmax<<<1, RB, 0, h->stream>>>(dcol, q.nz, psi_absmax);
    HIPCHK(hipGetLastError());
    return LBM_AXI_OK;
  });
}

int lbm_axi_pipe_nusselt(lbm_axi* h, int32_t inst, int32_t area, double* nu, double* T_b) {
  return guarded([&]() -> int {
    if (!h || inst < 0 || inst >= h->n_inst) return fail(LBM_AXI_EINVAL, "bad handle or instance");
    const lbm_axi_params& q = h->prm[inst];
    if (q.side_rmin != LBM_SIDE_AXIS || q.side_rmax != LBM_SIDE_WALL)
      return fail(LBM_AXI_EINVAL, "pipe Nusselt numbers need an axis at r_min and a wall at r_max");
    int64_t info[4];
    int rc = lbm_axi_info(h, inst, info);
    if (rc) return rc;
    const bool odd = (info[0] & 1) != 0;
    const size_t n = (size_t)q.nr * q.nz;
    void *dT = nullptr, *dU = nullptr, *dnu = nullptr, *dtb = nullptr;
    auto release_tmp = [&]() {
      (void)hipStreamSynchronize(h->stream);
      for (void* x : {dT, dU, dnu, dtb}) (void)hipFree(x);
    };
    if (hipMalloc(&dT, sizeof(float) * n) != hipSuccess || hipMalloc(&dU, sizeof(float) * n) != hipSuccess ||
        hipMalloc(&dnu, sizeof(double) * q.nz) != hipSuccess ||
        hipMalloc(&dtb, sizeof(double) * q.nz) != hipSuccess) {
      release_tmp();
      return fail(LBM_AXI_ENOMEM, "pipe Nusselt staging");
    }
    FieldOut fo{(float*)dU, nullptr, nullptr, (float*)dT, nullptr, nullptr};
    rc = launch_fields(h, inst, odd, fo);
    if (!rc) {
      k_pipe_nu<<<(q.nz + RB / 64 - 1) / (RB / 64), RB, 0, h->stream>>>(
          (const float*)dT, (const float*)dU, area ? 1 : 0, q.nr, q.nz, q.r0, (double*)dnu, (double*)dtb);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess && nu)
        e = hipMemcpyAsync(nu, dnu, sizeof(double) * q.nz, hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess && T_b)
        e = hipMemcpyAsync(T_b, dtb, sizeof(double) * q.nz, hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) rc = fail(LBM_AXI_EDEVICE, std::string("pipe Nusselt: ") + hipGetErrorString(e));
    }
    release_tmp();
    return rc;
  });
}

int lbm_axi_pattern_bandwidth(lbm_axi* h, int32_t reps, double* out) {
  return guarded([&]() -> int {
    if (!h || !out || reps < 1 || reps > 100000)
      return fail(LBM_AXI_EINVAL, "bad handle, output or reps out of [1, 100000]");
    HIPCHK(hipStreamSynchronize(h->stream));
    std::vector<int> st(h->n_inst);
    HIPCHK(hipMemcpy(st.data(), h->dstatus, sizeof(int) * h->n_inst, hipMemcpyDeviceToHost));
    // Algorithmic bytes of one step launch: per fluid node of the running
    // instances in the launch, 13 populations of the storage type and the
    // FP32 g_0 read and written, and the porosity read where it is a field.
    const double esz = h->storage == LBM_STORE_FP32 ? 4.0 : 2.0;
    double bytes = 0.0, arr = 0.0;
    for (int i = 0; i < h->n_inst; ++i) {
      const lbm_axi_params& q = h->prm[i];
      const InstDev& D = h->hdesc[i];
      arr += 14.0 * D.plane * esz + (h->storage == LBM_STORE_FP32 ? 0.0 : 4.0 * D.plane);
      if (st[i] != RUN || !(h->active.empty() || h->active[i])) continue;
      const double nrf = q.nr - (q.side_rmin == SIDE_WALL) - (q.side_rmax == SIDE_WALL);
      const double nzf = q.nz - (z_bounded(D) ? 2 : 0);
      bytes += nrf * nzf * (26.0 * esz + 8.0 + (D.phi ? 4.0 : 0.0));
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto timed = [&](auto&& launch, double& ms) -> int {
      launch();  // untimed first launch
      HIPCHK(hipEventRecord(e0, h->stream));
      for (int r = 0; r < reps; ++r) launch();
      HIPCHK(hipEventRecord(e1, h->stream));
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventSynchronize(e1));
      float f = 0.0f;
      HIPCHK(hipEventElapsedTime(&f, e0, e1));
      ms = f / reps;
      return LBM_AXI_OK;
    };
    double ms[3] = {0, 0, 0};
    int rc = LBM_AXI_OK;
    for (int par = 0; par < 2 && rc == LBM_AXI_OK; ++par) {
      const bool odd = par == 1;
      auto go = [&]() { (void)launch_pattern(h, odd, 0u); };
      rc = timed(go, ms[par]);
    }
    // plain stream: every instance's population array (and separate g_0 plane)
    // read and written in place, 16-byte words
    if (rc == LBM_AXI_OK) {
      auto go = [&]() {
        for (int i = 0; i < h->n_inst; ++i) {
          const InstDev& D = h->hdesc[i];
          const int64_t nw = 14 * D.plane * (int64_t)esz / 16;
          const unsigned nb = (unsigned)std::min<int64_t>((nw + RB - 1) / RB, 8192);
          k_stream_rw<<<nb, RB, 0, h->stream>>>((uint4*)D.pop, nw, 0u);
          if (h->storage != LBM_STORE_FP32)
            k_stream_rw<<<(unsigned)std::min<int64_t>((D.plane / 4 + RB - 1) / RB, 8192), RB, 0,
                          h->stream>>>((uint4*)D.g0, D.plane / 4, 0u);
        }
      };
      rc = timed(go, ms[2]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    out[0] = bytes / (ms[0] * 1e-3) / 1e9;
    out[1] = bytes / (ms[1] * 1e-3) / 1e9;
    out[2] = 2.0 * arr / (ms[2] * 1e-3) / 1e9;
    out[3] = bytes;
    return LBM_AXI_OK;
  });
}

int lbm_axi_lane_bandwidth(lbm_axi* h, int32_t reps, double* out) {
  return guarded([&]() -> int {
    if (!h || !out || reps < 1 || reps > 100000)
      return fail(LBM_AXI_EINVAL, "bad handle, output or reps out of [1, 100000]");
    HIPCHK(hipStreamSynchronize(h->stream));
    const int64_t esz = h->storage == LBM_STORE_FP32 ? 4 : 2;
    double arr = 0.0;
    for (const InstDev& D : h->hdesc) arr += 14.0 * D.plane * esz;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // every instance's population array (14 planes of a multiple-of-64 row
    // stride: a whole number of 16-byte words), read and written in place
    auto pass = [&](int w) {
      for (const InstDev& D : h->hdesc) {
        const int64_t n = 14 * D.plane * esz / w;
        const unsigned nb = (unsigned)std::min<int64_t>((n + RB - 1) / RB, 8192);
        if (w == 2) k_stream_lane<uint16_t><<<nb, RB, 0, h->stream>>>((uint16_t*)D.pop, n, 0u);
        if (w == 4) k_stream_lane<uint32_t><<<nb, RB, 0, h->stream>>>((uint32_t*)D.pop, n, 0u);
        if (w == 8) k_stream_lane<uint2><<<nb, RB, 0, h->stream>>>((uint2*)D.pop, n, 0u);
        if (w == 16) k_stream_lane<uint4><<<nb, RB, 0, h->stream>>>((uint4*)D.pop, n, 0u);
      }
    };
    int rc = LBM_AXI_OK;
    const int widths[4] = {2, 4, 8, 16};
    for (int q = 0; q < 4 && rc == LBM_AXI_OK; ++q) {
      rc = [&]() -> int {
        pass(widths[q]);  // untimed first pass
        HIPCHK(hipEventRecord(e0, h->stream));
        for (int r = 0; r < reps; ++r) pass(widths[q]);
        HIPCHK(hipEventRecord(e1, h->stream));
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventSynchronize(e1));
        float f = 0.0f;
        HIPCHK(hipEventElapsedTime(&f, e0, e1));
        out[q] = 2.0 * arr / (f / reps * 1e-3) / 1e9;
        return LBM_AXI_OK;
      }();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
  });
}

int lbm_axi_set_timing(lbm_axi* h, int32_t on) {
  return guarded([&]() -> int {
    if (!h) return fail(LBM_AXI_EINVAL, "null handle");
    if (on && !h->timing) {
      double ms;
      int64_t nl;
      int rc = lbm_axi_kernel_time(h, &ms, &nl);
      if (rc) return rc;
      h->timed_ms = 0.0;
      h->timed_launches = 0;
    }
    h->timing = on != 0;
    return LBM_AXI_OK;
  });
}

int lbm_axi_kernel_time(lbm_axi* h, double* total_ms, int64_t* launches) {
  return guarded([&]() -> int {
    if (!h) return fail(LBM_AXI_EINVAL, "null handle");
    if (!h->ev.empty()) {
      HIPCHK(hipEventSynchronize(h->ev.back().second));
      for (auto& e : h->ev) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e.first, e.second));
        h->timed_ms += ms;
        h->timed_launches += 1;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
      h->ev.clear();
    }
    if (total_ms) *total_ms = h->timed_ms;
    if (launches) *launches = h->timed_launches;
    return LBM_AXI_OK;
  });
}

}  // extern "C"
