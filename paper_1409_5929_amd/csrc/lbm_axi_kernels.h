// Step-kernel templates of the library and the launch interface of their
// 16-bit instantiations.  The FP32 kernels are instantiated in lbm_axi.hip,
// the FP16 and BF16 kernels in lbm_axi_s16.hip: compiled apart, each storage
// type's kernels get the schedule that measured fastest for it (the compiler
// shapes shared inlined code by what else the file holds).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_axi_dev.h"

namespace lbmaxi {

constexpr int BX = LANES_R;  // lanes along r
constexpr int BY = 4;        // waves per block, interleaved along z

// 16-bit steps ask for at least 4 waves per SIMD (at most 128 VGPRs): some
// variants land one register above that otherwise and lose a quarter of
// their waves (measured: the 1024-instance sweep 1.15 against 1.24 ms per
// step).
template <typename S, bool ODD, int MODE, bool BUF, bool WL = false>
__global__ __launch_bounds__(BX* BY) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 2 ? 4 : 1))) void k_step(const InstDev* __restrict__ descs,
                                                 const int4* __restrict__ tiles,
                                                 const int* __restrict__ status, int kz,
                                                 int mac_slot, FieldOut fo, uint32_t seed,
                                                 const long long* __restrict__ clk, int off) {
  // Inside a captured step graph the time level comes from the device clock
  // (set before every replay) plus the step's offset in the graph.
  if (clk) seed = step_seed(*clk + off);
  const int4 tl = tiles[blockIdx.x];
  if (tl.x < 0) return;
  if (MODE != MODE_FIELDS && status[tl.x] != RUN) return;
  const InstDev D = descs[tl.x];
  // A packed tile (tl.w = 1) covers 32 columns: lanes 32..63 take the z strip
  // after lanes 0..31's (a row's last, at most half-wide column tile).
  const int half = tl.w ? (int)(threadIdx.x >> 5) : 0;
  const int jt = tl.y + (tl.w ? (int)(threadIdx.x & 31) : (int)threadIdx.x);
  if (jt >= D.nr) return;
  // With wall lanes (WL) a radial wall lane (column 0 or nr - 1 of a no-slip
  // side) works on its owner's column j and writes its own wall node
  // (wall_lane_inputs) when it shares the owner's wave; otherwise, and without
  // wall lanes, the owner computes the wall node and the wall lane idles.
  int wl = 0;
  if constexpr (WL && MODE != MODE_FIELDS) {
    wl = (D.side_rmin == SIDE_WALL && jt == 0) ? 1 : (D.side_rmax == SIDE_WALL && jt == D.nr - 1) ? -1 : 0;
    if (wl < 0 && !wall_lane_rmax(D)) return;
  } else {
    if ((D.side_rmin == SIDE_WALL && jt == 0) || (D.side_rmax == SIDE_WALL && jt == D.nr - 1)) return;
  }
  const int j = jt + wl;
  const RowC R = make_row(D, j);
  const bool zwall = z_bounded(D);
  // Fluid nodes of this thread's strip: k = kbeg, kbeg + BY, ... < kend.
  const int k0 = tl.z + (int)threadIdx.y + half * BY * kz;
  int kbeg = k0, kend = min(k0 + BY * kz, D.nz);
  if (zwall) {
    if (kbeg == 0) kbeg += BY;
    if (kend == D.nz && (D.nz - 1 - k0) % BY == 0) kend = D.nz - 1;  // top wall row in this strip
  }
  // The two-stage pipeline below pays off only for the FP32 odd step: there
  // the loads are scattered over three rows and the registers allow it (even
  // steps would exceed 256 VGPRs; 16-bit steps would lose a wave per SIMD).
  if (MODE == MODE_FIELDS || !ODD || sizeof(S) != 4) {
    for (int k = kbeg; k < kend; k += BY) node_update<S, ODD, MODE, BUF, WL>(D, R, j, k, mac_slot, fo, seed, wl);
    return;
  }
  if (kbeg >= kend) return;
  // Two-stage pipeline: the next node's loads are in flight while this node
  // is updated (each slot belongs to one node of the step, so the order of
  // one thread's loads and stores across its nodes does not matter).
  float s[9], t[5], ph;
  node_load<S, ODD, BUF>(D, R, j, kbeg, s, t, ph);
  for (int k = kbeg; k < kend; k += BY) {
    float sn[9], tn[5], phn = 0.0f;
    const bool more = k + BY < kend;
    if (more) node_load<S, ODD, BUF>(D, R, j, k + BY, sn, tn, phn);
    node_update_loaded<S, ODD, MODE, BUF, WL>(D, R, j, k, mac_slot, fo, seed, s, t, ph, wl);
    if (!more) break;
#pragma unroll
    for (int q = 0; q < 9; ++q) s[q] = sn[q];
#pragma unroll
    for (int q = 0; q < 5; ++q) t[q] = tn[q];
    ph = phn;
  }
}

// Streaming-ceiling probe of the step: the step's launch (tiles, strips of
// kz nodes, addressing) and its loads and stores, with no arithmetic
// (pattern_store); two nodes of a strip are in flight at a time.
template <typename S, bool ODD, bool BUF>
__global__ __launch_bounds__(BX* BY) void k_pattern(const InstDev* __restrict__ descs,
                                                    const int4* __restrict__ tiles,
                                                    const int* __restrict__ status, int kz,
                                                    uint32_t key) {
  const int4 tl = tiles[blockIdx.x];
  if (tl.x < 0 || status[tl.x] != RUN) return;
  const InstDev D = descs[tl.x];
  const int half = tl.w ? (int)(threadIdx.x >> 5) : 0;  // packed tile: see k_step
  const int j = tl.y + (tl.w ? (int)(threadIdx.x & 31) : (int)threadIdx.x);
  if (j >= D.nr) return;
  if ((D.side_rmin == SIDE_WALL && j == 0) || (D.side_rmax == SIDE_WALL && j == D.nr - 1)) return;
  const RowC R = make_row(D, j);
  const int k0 = tl.z + (int)threadIdx.y + half * BY * kz;
  int kbeg = k0, kend = min(k0 + BY * kz, D.nz);
  if (z_bounded(D)) {
    if (kbeg == 0) kbeg += BY;
    if (kend == D.nz && (D.nz - 1 - k0) % BY == 0) kend = D.nz - 1;
  }
  for (int k = kbeg; k < kend; k += 2 * BY) {
    float s[9], t[5], ph, s2[9], t2[5], ph2 = 0.0f;
    const bool two = k + BY < kend;
    node_load<S, ODD, BUF>(D, R, j, k, s, t, ph);
    if (two) node_load<S, ODD, BUF>(D, R, j, k + BY, s2, t2, ph2);
    pattern_store<S, ODD, BUF>(D, R, j, k, s, t, ph, key);
    if (two) pattern_store<S, ODD, BUF>(D, R, j, k + BY, s2, t2, ph2, key);
  }
}

// Start state of one instance from (u_z, u_r, T) fields (nr x nz each, in
// that order) or from rest at T_init.
template <typename S>
__global__ __launch_bounds__(BX* BY) void k_init(const InstDev* __restrict__ descs,
                                                 const int4* __restrict__ tiles, int kz,
                                                 const float* __restrict__ init, int inst) {
  const int4 tl = tiles[blockIdx.x];
  if (tl.x != inst) return;
  const InstDev D = descs[inst];
  const int j = tl.y + (int)threadIdx.x;
  if (j >= D.nr) return;
  const int64_t n = (int64_t)D.nr * D.nz;
  for (int i = 0; i < kz; ++i) {
    const int k = tl.z + (int)threadIdx.y + BY * i;
    if (k >= D.nz) break;
    const int64_t o = (int64_t)k * D.nr + j;
    init_node<S>(D, j, k, init[o], init[n + o], init[2 * n + o]);
  }
}

// Start state without an init field: rest, uniform T_init.
template <typename S>
__global__ __launch_bounds__(BX* BY) void k_init_uniform(const InstDev* __restrict__ descs,
                                                         const int4* __restrict__ tiles, int kz,
                                                         float T_init, int inst) {
  const int4 tl = tiles[blockIdx.x];
  if (tl.x != inst) return;
  const InstDev D = descs[inst];
  const int j = tl.y + (int)threadIdx.x;
  if (j >= D.nr) return;
  for (int i = 0; i < kz; ++i) {
    const int k = tl.z + (int)threadIdx.y + BY * i;
    if (k >= D.nz) break;
    init_node<S>(D, j, k, 0.0f, 0.0f, T_init);
  }
}


// Launch description of a step-shaped kernel over a tile list.
struct StepLaunch {
  const InstDev* descs;
  const int4* tiles;
  const int* status;
  int ntiles;
  int kz;
  int lds_bytes;
  hipStream_t stream;
};

// Launches of one storage type's kernels (instantiated by whichever file
// calls them).  Step kernels: even or odd parity of the AA step, plain or
// with the check's macroscopic output (mode), buffer or flat addressing
// (BUF), with or without wall lanes (WL).
template <typename S, bool BUF, bool WL>
hipError_t launch_step_t(bool odd, int mode, const StepLaunch& L, int mac_slot, uint32_t seed,
                         const long long* clk, int off) {
  const dim3 blk(BX, BY);
  const FieldOut fo{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  if (!odd) {
    if (mode == MODE_STEP)
      k_step<S, false, MODE_STEP, BUF, WL><<<L.ntiles, blk, L.lds_bytes, L.stream>>>(L.descs, L.tiles, L.status, L.kz, mac_slot, fo, seed, clk, off);
    else
      k_step<S, false, MODE_STEP_MACRO, BUF, WL><<<L.ntiles, blk, L.lds_bytes, L.stream>>>(L.descs, L.tiles, L.status, L.kz, mac_slot, fo, seed, clk, off);
  } else {
    if (mode == MODE_STEP)
      k_step<S, true, MODE_STEP, BUF, WL><<<L.ntiles, blk, L.lds_bytes, L.stream>>>(L.descs, L.tiles, L.status, L.kz, mac_slot, fo, seed, clk, off);
    else
      k_step<S, true, MODE_STEP_MACRO, BUF, WL><<<L.ntiles, blk, L.lds_bytes, L.stream>>>(L.descs, L.tiles, L.status, L.kz, mac_slot, fo, seed, clk, off);
  }
  return hipGetLastError();
}
template <typename S, bool BUF>
hipError_t launch_step_b(bool wall_lanes, bool odd, int mode, const StepLaunch& L, int mac_slot,
                         uint32_t seed, const long long* clk, int off) {
  return wall_lanes ? launch_step_t<S, BUF, true>(odd, mode, L, mac_slot, seed, clk, off)
                    : launch_step_t<S, BUF, false>(odd, mode, L, mac_slot, seed, clk, off);
}
// Macroscopic fields of one instance (no population writes).
template <typename S>
hipError_t launch_fields_t(bool odd, const StepLaunch& L, const FieldOut& fo) {
  const dim3 blk(BX, BY);
  if (!odd)
    k_step<S, false, MODE_FIELDS, false><<<L.ntiles, blk, 0, L.stream>>>(L.descs, L.tiles, L.status, L.kz, 0, fo, 0u, nullptr, 0);
  else
    k_step<S, true, MODE_FIELDS, false><<<L.ntiles, blk, 0, L.stream>>>(L.descs, L.tiles, L.status, L.kz, 0, fo, 0u, nullptr, 0);
  return hipGetLastError();
}
// Streaming-ceiling probe with the step's launch and addressing.
template <typename S, bool BUF>
hipError_t launch_pattern_t(bool odd, const StepLaunch& L, uint32_t key) {
  const dim3 blk(BX, BY);
  if (!odd)
    k_pattern<S, false, BUF><<<L.ntiles, blk, L.lds_bytes, L.stream>>>(L.descs, L.tiles, L.status, L.kz, key);
  else
    k_pattern<S, true, BUF><<<L.ntiles, blk, L.lds_bytes, L.stream>>>(L.descs, L.tiles, L.status, L.kz, key);
  return hipGetLastError();
}
// Start state of instance inst (fields, or rest at T_init when dinit is null).
template <typename S>
hipError_t launch_init_t(const StepLaunch& L, const float* dinit, float T_init, int inst) {
  const dim3 blk(BX, BY);
  if (dinit)
    k_init<S><<<L.ntiles, blk, 0, L.stream>>>(L.descs, L.tiles, L.kz, dinit, inst);
  else
    k_init_uniform<S><<<L.ntiles, blk, 0, L.stream>>>(L.descs, L.tiles, L.kz, T_init, inst);
  return hipGetLastError();
}

// FP16 / BF16 launches (lbm_axi_s16.hip); storage is LBM_STORE_FP16 or
// LBM_STORE_BF16.  Each returns the launch's hipError_t.
hipError_t launch_step_s16(int storage, bool buf, bool wall_lanes, bool odd, int mode, const StepLaunch& L,
                           int mac_slot, uint32_t seed, const long long* clk, int off);
hipError_t launch_fields_s16(int storage, bool odd, const StepLaunch& L, const FieldOut& fo);
hipError_t launch_pattern_s16(int storage, bool buf, bool odd, const StepLaunch& L, uint32_t key);
hipError_t launch_init_s16(int storage, const StepLaunch& L, const float* dinit, float T_init, int inst);

}  // namespace lbmaxi
