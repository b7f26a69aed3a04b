// FP16 and BF16 instantiations of the step kernels (lbm_axi_kernels.h), in a
// file of their own so that the compiler schedules them apart from the FP32
// kernels: here the branch into the owners' wall-node work is marked
// unlikely, which keeps that work out of every fluid node's update in the
// 16-bit steps (measured: FP16 8192^2 0.920 -> 0.885 ms per step, the
// 1024-instance sweep 1.206 -> 1.146 ms) but slows the FP32 steps (3 %).
#define LBM_OWNER_WALLS_UNLIKELY 1

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "../../include/lbm_axi.h"
#include "lbm_axi_kernels.h"

namespace lbmaxi {

template <typename S>
hipError_t step_s(bool buf, bool wl, bool odd, int mode, const StepLaunch& L, int slot, uint32_t seed,
                  const long long* clk, int off) {
  return buf ? launch_step_b<S, true>(wl, odd, mode, L, slot, seed, clk, off)
             : launch_step_b<S, false>(wl, odd, mode, L, slot, seed, clk, off);
}

hipError_t launch_step_s16(int storage, bool buf, bool wall_lanes, bool odd, int mode, const StepLaunch& L,
                           int mac_slot, uint32_t seed, const long long* clk, int off) {
  if (storage == LBM_STORE_FP16) return step_s<__half>(buf, wall_lanes, odd, mode, L, mac_slot, seed, clk, off);
  return step_s<__hip_bfloat16>(buf, wall_lanes, odd, mode, L, mac_slot, seed, clk, off);
}

hipError_t launch_fields_s16(int storage, bool odd, const StepLaunch& L, const FieldOut& fo) {
  if (storage == LBM_STORE_FP16) return launch_fields_t<__half>(odd, L, fo);
  return launch_fields_t<__hip_bfloat16>(odd, L, fo);
}

hipError_t launch_pattern_s16(int storage, bool buf, bool odd, const StepLaunch& L, uint32_t key) {
  if (storage == LBM_STORE_FP16)
    return buf ? launch_pattern_t<__half, true>(odd, L, key) : launch_pattern_t<__half, false>(odd, L, key);
  return buf ? launch_pattern_t<__hip_bfloat16, true>(odd, L, key)
             : launch_pattern_t<__hip_bfloat16, false>(odd, L, key);
}

hipError_t launch_init_s16(int storage, const StepLaunch& L, const float* dinit, float T_init, int inst) {
  if (storage == LBM_STORE_FP16) return launch_init_t<__half>(L, dinit, T_init, inst);
  return launch_init_t<__hip_bfloat16>(L, dinit, T_init, inst);
}

}  // namespace lbmaxi
