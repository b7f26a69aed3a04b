// Per-node update of the axisymmetric D2Q9-MRT / D2Q5 lattice Boltzmann step
// (Liu, He, Li, arXiv:1409.5929, Secs. 3.1-3.2), shared by the step, start
// and field kernels of lbm_axi.hip.
//
// Storage.  One array of 14 planes per instance (f_0..f_8, then g_0..g_4),
// each plane [nz][stride] with r fastest, updated in place with the AA
// pattern: at even time levels the slot (i, x) holds the population f_i that
// has arrived at x; an even step reads a node's own slots and writes f_i^+ to
// its own slot opposite(i); an odd step reads f_i from slot opposite(i) of
// x - e_i and writes f_i^+ to slot i of x + e_i.  Every thread writes exactly
// the slots it read, so the update needs no second array and no barrier.
//
// Values.  The populations are r-weighted (Eq. 17, Eq. 26): f_i = r fhat_i.
// A slot holds the deviation of fhat_i from the scheme's quiescent state
// (rho = 1, u = 0, only the axisymmetric term a_r acting), in the frame of
// the node that wrote it (the source x - e_i of an arriving population).
// That state is fhat_i = w_i (1 + e_ir / (2 r)) after collision and
// w_i (1 - e_ir / (2 r)) before it; streaming maps the first onto the second
// exactly (r_src = r - e_ir), so the reader only rescales the deviation,
// d_i = (r_src / r) s_i, and the collision maps zero deviations onto zero.
// FP32 thus keeps its relative precision at any r, also next to the axis,
// and the same representation serves FP16/BF16 storage (times a power of
// two, rounded stochastically).  Temperature slots hold g_i - wt_i T_s for a
// storage shift T_s; the resting temperature population g_0 (which never
// streams) lives in an FP32 plane of its own in every storage type.
//
// Axis.  With an axis at r_min the mirror row j = -1 is never stored: its
// slot q at (-1, k) is the slot q* (e_r reversed) of (0, k).  In the writer's
// frame the odd mirror f_i(-r) = -f_i*(r) of the r-weighted populations is
// the plain copy fhat_i(-r) = fhat_i*(r), so the alias needs no arithmetic;
// the reader's rescaling with r_src = -1/2 restores the sign.
//
// Walls.  Boundary nodes (rows 0 / nr-1, columns 0 / nz-1: no-slip walls,
// or an inlet and an outlet column) are reconstructed by non-equilibrium
// extrapolation (Sec. 4) from a fluid neighbour B that owns them (normal
// neighbour; diagonal one for corners), each with its own density, velocity
// and temperature.  B's thread computes the boundary node's post-collision
// populations from its own registers and writes the ones that stream into
// fluid nodes, also through the axis mirror, to the AA slots the boundary
// node would have written.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbmaxi {

enum { SIDE_WALL = 0, SIDE_AXIS = 1, SIDE_PERIODIC = 2, SIDE_FLOW = 3 };
enum { THERM_FIXED = 0, THERM_ADIABATIC = 1, THERM_FLUX = 2 };
enum { RUN = 0, CONVERGED = 1, DIVERGED = 2, STALLED = 3 };
enum { MODE_STEP = 0, MODE_STEP_MACRO = 1, MODE_FIELDS = 2 };
enum { MASK_RMIN = 1, MASK_RMAX = 2, MASK_ZMIN = 4, MASK_ZMAX = 8, MASK_AXIS = 16 };

// Lanes of a step wave along r: the step's tiles start at multiples of it,
// so columns c and c' share a wave when c / LANES_R == c' / LANES_R.
constexpr int LANES_R = 64;

// c_s^2 of D2Q9 (text after Eq. 25); weights of Eq. (32); D2Q5 weights of
// Eq. (36) with wt_0 = 3/5 and c_sT^2 = 1/5.
constexpr float CS2 = (float)(1.0 / 3.0);
constexpr float W0 = (float)(4.0 / 9.0), W1 = (float)(1.0 / 9.0), W5 = (float)(1.0 / 36.0);
constexpr float WT0 = (float)0.6, WT1 = (float)0.1;

// Everything a kernel needs about one instance (uniform across a block, so
// the compiler keeps it in scalar registers).
struct InstDev {
  int32_t nr, nz, stride, pad0;
  int64_t plane;  // stride * nz
  int32_t side_rmin, side_rmax, side_z;
  int32_t therm_rmin, therm_rmax, therm_z;
  int32_t src_printed;
  int32_t phi_mode;  // 0 uniform, 1 field with Ergun F_phi, 2 field with constant F_phi
  void* pop;         // 14 planes
  uint32_t pop_bytes;  // size of pop in bytes when below 4 GiB (buffer addressing), else 0
  float* g0;         // plane of g_0 - wt_0 T_s in FP32 for every storage type: plane 9 of
                     // pop in FP32, its own plane otherwise (g_0 never streams and carries
                     // most of T, so 16 bits there would dominate the error of T)
  const float* phi;  // [nz][stride] porosity field or null
  float* mac[2];     // two check buffers, 3 planes each: u_z, u_r, T
  float r0, T_ref, gbeta, accel_r, accel_z;
  float T_s;          // temperature storage shift
  float az_s;         // accel_z + gbeta (T_s - T_ref): buoyancy offset in theta = T - T_s
  float c_tau;        // c_s^2 (tau_nu - 1/2)
  float s_e, s_eps, s_j, s_q, s_nu;  // rates of Eq. (23)
  float phiu, cD, cF; // uniform porosity, phi nu / K, phi F_phi / sqrt(K)
  float C1, C2, C3;   // porosity-field coefficients of cD and cF
  float tau_T, omc;   // omc = 1 / (tau_T + 1/2)
  float T_rmin, T_rmax, T_zmin, T_zmax;
  float st_scale, st_inv;  // storage scale 2^shift and its inverse
  float q_rmin, q_rmax;    // q'/k of isoflux radial walls
  int32_t qk_lo, qk_hi;    // heated columns qk_lo..qk_hi of an isoflux wall
  float u_in;              // inlet axial velocity with inlet/outlet columns
};

// Optional outputs of the field kernel ([nz][nr], unpadded).
struct FieldOut {
  float *uz, *ur, *p, *T;
  uint8_t* mask;
  float* drho;  // rho - 1
};

// ---- storage types --------------------------------------------------------
// st() rounds to nearest even; st_sr() rounds stochastically with 32 random
// bits r: the FP32 value is rounded away from zero with probability equal to
// its distance from the 16-bit value below (in magnitude) over the 16-bit
// spacing, so that the stored value is unbiased.  Deterministic rounding lets
// a slowly varying population round back to its old value step after step,
// so a run freezes short of its steady state.  On the device this is one
// gfx950 conversion instruction (v_cvt_sr_f16_f32 / v_cvt_sr_bf16_f32, which
// take the random bits as an operand).  The host version adds the random
// bits to the FP32 bit pattern below the 16-bit mantissa and truncates (the
// carry moves into the next mantissa step or exponent); there, results in
// the FP16 subnormal range (|v sc| < 2^-14) are rounded to nearest after.
typedef _Float16 lbm_h2 __attribute__((ext_vector_type(2)));
typedef __bf16 lbm_b2 __attribute__((ext_vector_type(2)));
template <typename S>
struct Store;
template <>
struct Store<float> {
  __host__ __device__ static inline float ld(const float* p, int64_t i, float) { return p[i]; }
  __host__ __device__ static inline void st(float* p, int64_t i, float v, float) { p[i] = v; }
  __host__ __device__ static inline void st_sr(float* p, int64_t i, float v, float, uint32_t) {
    p[i] = v;
  }
};
template <>
struct Store<__half> {
  __host__ __device__ static inline float ld(const __half* p, int64_t i, float inv) {
    return __half2float(p[i]) * inv;
  }
  __host__ __device__ static inline void st(__half* p, int64_t i, float v, float sc) {
    p[i] = __float2half_rn(v * sc);
  }
  __host__ __device__ static inline void st_sr(__half* p, int64_t i, float v, float sc,
                                               uint32_t r) {
#if defined(__HIP_DEVICE_COMPILE__)
    const lbm_h2 h = __builtin_amdgcn_cvt_sr_f16_f32(lbm_h2{0, 0}, v * sc, r, false);
    p[i] = __builtin_bit_cast(__half, h[0]);
#else
    const uint32_t b = (__float_as_uint(v * sc) + (r >> 19)) & 0xFFFFE000u;  // 13 dropped bits
    p[i] = __float2half_rn(__uint_as_float(b));
#endif
  }
};
template <>
struct Store<__hip_bfloat16> {
  __host__ __device__ static inline float ld(const __hip_bfloat16* p, int64_t i, float inv) {
    return __bfloat162float(p[i]) * inv;
  }
  __host__ __device__ static inline void st(__hip_bfloat16* p, int64_t i, float v, float sc) {
    p[i] = __float2bfloat16(v * sc);
  }
  __host__ __device__ static inline void st_sr(__hip_bfloat16* p, int64_t i, float v, float sc,
                                               uint32_t r) {
#if defined(__HIP_DEVICE_COMPILE__)
    const lbm_b2 h = __builtin_amdgcn_cvt_sr_bf16_f32(lbm_b2{0, 0}, v * sc, r, false);
    p[i] = __builtin_bit_cast(__hip_bfloat16, h[0]);
#else
    const uint32_t b = (__float_as_uint(v * sc) + (r >> 16)) & 0xFFFF0000u;  // 16 dropped bits
    p[i] = __float2bfloat16(__uint_as_float(b));
#endif
  }
};

// Random bits for stochastic rounding: a 32-bit integer hash (xorshift-
// multiply finaliser, Wellons' "lowbias32" constants) of the step seed and
// the node's offset seeds a per-node linear congruential stream (Knuth's
// MMIX multiplier and increment, mod 2^32).  The roundings use only the
// high 16 bits of their random operand (13 for FP16), so each state feeds
// two stores: the state itself, then its low half moved up.
__host__ __device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
// Population layout of node offset o (a multiple-of-64 row stride times z,
// planes of pl elements).  Slots 0..8 hold f_0..f_8, slots 10..13 g_1..g_4;
// g_0 is slot 9 in FP32 storage and an FP32 plane of its own otherwise.
// FP32: slot q at element q pl + o.  16-bit storage: the axial D2Q9 slot
// q = 1..4 and the D2Q5 slot q + 9 share a 32-bit word (low and high half):
// the AA step reads and writes these two at the same node in both parities,
// so one 32-bit access moves both.  Word o of pair plane a = q - 1 sits at
// elements (5 + 2a) pl + 2o; slots 0, 5, 6, 7, 8 keep 16-bit planes 0..4.
// (Measured: an in-place stream moves 3.0 TB/s with 2-byte lanes against
// 4.7-5.0 TB/s with 4-byte lanes; the memory pipeline is bound by
// instructions, not bytes, at 2 bytes per lane.)
template <typename S>
__host__ __device__ inline int64_t slot_elem(int q, int64_t o, int64_t pl) {
  if constexpr (sizeof(S) == 4) {
    return q * pl + o;
  } else {
    if (q >= 1 && q <= 4) return (3 + 2 * q) * pl + 2 * o;
    if (q >= 10) return (2 * q - 15) * pl + 2 * o + 1;
    return (q == 0 ? 0 : q - 4) * pl + o;
  }
}

// ---- population access --------------------------------------------------
// PopAcc<S, false>: flat addressing through a pointer (64-bit addresses per
// lane).  PopAcc<S, true>: buffer addressing, one descriptor in scalar
// registers per instance and 32-bit byte offsets per lane (half the address
// registers; the hardware also drops accesses outside the array), usable when
// the population array is below 4 GiB.  The hardware takes the record count
// and the offsets as unsigned 32-bit values; the builtins declare them int,
// so values of 2^31 and above pass as their bit patterns.
// ld / st: slot q of node o.  ld_pair / st_pair: slots a + 1 and a + 10 of
// node o (a = 0..3), one 32-bit access in 16-bit storage; the two stochastic
// roundings fill the low and the high half of the stored word.
template <typename S>
__device__ inline uint32_t pack_sr(float f, float g, uint32_t rf, uint32_t rg) {
  if constexpr (std::is_same<S, __half>::value) {
    lbm_h2 h = __builtin_amdgcn_cvt_sr_f16_f32(lbm_h2{0, 0}, f, rf, false);
    h = __builtin_amdgcn_cvt_sr_f16_f32(h, g, rg, true);
    return __builtin_bit_cast(uint32_t, h);
  } else {
    lbm_b2 h = __builtin_amdgcn_cvt_sr_bf16_f32(lbm_b2{0, 0}, f, rf, false);
    h = __builtin_amdgcn_cvt_sr_bf16_f32(h, g, rg, true);
    return __builtin_bit_cast(uint32_t, h);
  }
}
template <typename S>
__device__ inline void unpack(uint32_t w, float inv, float& f, float& g) {
  if constexpr (std::is_same<S, __half>::value) {
    const lbm_h2 h = __builtin_bit_cast(lbm_h2, w);
    f = (float)h[0] * inv;
    g = (float)h[1] * inv;
  } else {
    f = __uint_as_float(w << 16) * inv;
    g = __uint_as_float(w & 0xFFFF0000u) * inv;
  }
}

template <typename S, bool BUF>
struct PopAcc;
template <typename S>
struct PopAcc<S, false> {
  S* P;
  int64_t pl;
  float inv, sc;
  __host__ __device__ explicit PopAcc(const InstDev& D)
      : P((S*)D.pop), pl(D.plane), inv(D.st_inv), sc(D.st_scale) {}
  __host__ __device__ float ld(int q, int64_t o) const { return Store<S>::ld(P, slot_elem<S>(q, o, pl), inv); }
  __host__ __device__ void st(int q, int64_t o, float v, uint32_t r) const {
    Store<S>::st_sr(P, slot_elem<S>(q, o, pl), v, sc, r);
  }
  __host__ __device__ void ld_pair(int a, int64_t o, float& f, float& g) const {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(S) == 2) {
      unpack<S>(((const uint32_t*)P)[(int64_t)(5 + 2 * a) * (pl >> 1) + o], inv, f, g);
      return;
    }
#endif
    f = ld(a + 1, o);
    g = ld(a + 10, o);
  }
  __host__ __device__ void st_pair(int a, int64_t o, float f, float g, uint32_t rf, uint32_t rg) const {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(S) == 2) {
      ((uint32_t*)P)[(int64_t)(5 + 2 * a) * (pl >> 1) + o] = pack_sr<S>(f * sc, g * sc, rf, rg);
      return;
    }
#endif
    st(a + 1, o, f, rf);
    st(a + 10, o, g, rg);
  }
};
template <typename S>
struct PopAcc<S, true> {
#if defined(__HIP_DEVICE_COMPILE__)
  __amdgpu_buffer_rsrc_t rs;
#endif
  int64_t pl;
  float inv, sc;
  __host__ __device__ explicit PopAcc(const InstDev& D) : pl(D.plane), inv(D.st_inv), sc(D.st_scale) {
#if defined(__HIP_DEVICE_COMPILE__)
    rs = __builtin_amdgcn_make_buffer_rsrc(D.pop, (short)0, (int)(uint32_t)D.pop_bytes, 0x00020000);
#endif
  }
  __host__ __device__ float ld(int q, int64_t o) const {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t off = (uint32_t)slot_elem<S>(q, o, pl) * (uint32_t)sizeof(S);
    if constexpr (std::is_same<S, float>::value) {
      return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
    } else {
      const uint16_t b = (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(rs, (int)off, 0, 0);
      if constexpr (std::is_same<S, __half>::value)
        return __half2float(__builtin_bit_cast(__half, b)) * inv;
      else
        return __uint_as_float((uint32_t)b << 16) * inv;
    }
#else
    (void)q;
    (void)o;
    return 0.0f;
#endif
  }
  __host__ __device__ void st(int q, int64_t o, float v, uint32_t r) const {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t off = (uint32_t)slot_elem<S>(q, o, pl) * (uint32_t)sizeof(S);
    if constexpr (std::is_same<S, float>::value) {
      (void)r;
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, (int)off, 0, 0);
    } else if constexpr (std::is_same<S, __half>::value) {
      const lbm_h2 h = __builtin_amdgcn_cvt_sr_f16_f32(lbm_h2{0, 0}, v * sc, r, false);
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h[0]), rs, (int)off, 0, 0);
    } else {
      const lbm_b2 h = __builtin_amdgcn_cvt_sr_bf16_f32(lbm_b2{0, 0}, v * sc, r, false);
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h[0]), rs, (int)off, 0, 0);
    }
#else
    (void)q;
    (void)o;
    (void)v;
    (void)r;
#endif
  }
  __host__ __device__ void ld_pair(int a, int64_t o, float& f, float& g) const {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(S) == 2) {
      const uint32_t off = (uint32_t)((int64_t)(5 + 2 * a) * pl + 2 * o) * 2u;
      unpack<S>((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0), inv, f, g);
      return;
    }
#endif
    f = ld(a + 1, o);
    g = ld(a + 10, o);
  }
  __host__ __device__ void st_pair(int a, int64_t o, float f, float g, uint32_t rf, uint32_t rg) const {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(S) == 2) {
      const uint32_t off = (uint32_t)((int64_t)(5 + 2 * a) * pl + 2 * o) * 2u;
      __builtin_amdgcn_raw_buffer_store_b32(pack_sr<S>(f * sc, g * sc, rf, rg), rs, (int)off, 0, 0);
      return;
    }
#endif
    st(a + 1, o, f, rf);
    st(a + 10, o, g, rg);
  }
};

// Random bits of time level n (one value per step, shared by all nodes).
__host__ __device__ inline uint32_t step_seed(long long n) {
  return mix32((uint32_t)n * 0x9E3779B9u + (uint32_t)((unsigned long long)n >> 32));
}
struct Dither {
  uint32_t s;
  bool low = false;  // the low half of s is still unused
  __host__ __device__ explicit Dither(uint32_t seed) : s(seed) {}
  __host__ __device__ inline uint32_t next() {
    if (low) {
      low = false;
      return s << 16;
    }
    s = s * 1664525u + 1013904223u;
    low = true;
    return s;
  }
};

// Offset of row k in a plane (64-bit: planes of large grids pass 2^31).
__host__ __device__ inline int64_t row_off(int k, int stride) { return (int64_t)k * stride; }

// ---- per-column constants (r is fixed along a thread's z loop) -------------
struct RowC {
  float r, inv_r;
  float rp, op1, op5;  // sources of e_r = +1 populations: ratio r_src / r, offsets
  float rm, om1, om5;  // sources of e_r = -1 populations (offsets vanish unless r wraps)
  float lr0b;          // (1 + c_s^2 (tau - 1/2) / r^2) / 2, Eq. (30) divided by r
  float hcs2r;         // c_s^2 / (2 r), Eq. (29) divided by r rho
  float ar0, ar1;      // a_r = ar0 - ar1 u_r, Eq. (25)
  float omT1, omT3;    // D2Q5 rates for e_r = +1, -1 (after Eq. 33)
  int cm, cp;          // column of x - e_r for e_r = +1 / -1 sources (after wrap or alias)
  bool mir;            // x - (1, 0) is the axis mirror row
};

__host__ __device__ inline RowC make_row(const InstDev& D, int j) {
  // Row j sits at r = r0 + j, exact in FP64.  The streaming rescale factors
  // r_src / r and the wrap offsets carry every arriving population, and mass
  // is conserved only if they match the radii the neighbouring rows use, so
  // they are FP64 quotients rounded once.  The other constants take FP32 from
  // the correctly rounded 1 / r: their rounding is one more FP32 rounding of
  // the update (measured against the oracle: no change beyond 1e-7).
  RowC R;
  const double rd = (double)D.r0 + j;
  const bool rper = D.side_rmin == SIDE_PERIODIC;
  const bool wrap_p = j == 0 && rper, wrap_m = j == D.nr - 1 && rper;
  R.cm = j - 1;
  R.cp = j + 1;
  R.mir = false;
  if (j == 0 && D.side_rmin == SIDE_AXIS) {
    R.cm = 0;
    R.mir = true;  // source radius r - 1 = -1/2 is the mirror row itself
  }
  if (wrap_p) R.cm = D.nr - 1;
  if (wrap_m) R.cp = 0;
  const double src_p = wrap_p ? (double)D.r0 + (D.nr - 1) : rd - 1.0;
  const double src_m = wrap_m ? (double)D.r0 : rd + 1.0;
  // d = (r_src / r) s + w (r_src - r + e_r) / r: the offset is zero unless
  // the source sits across a radial wrap (r_src != r - e_r).
  const double invd = 1.0 / rd;
  R.rp = (float)(src_p * invd);
  R.rm = (float)(src_m * invd);
  R.op1 = R.op5 = R.om1 = R.om5 = 0.0f;
  if (wrap_p) {
    const double gp = (src_p - rd + 1.0) * invd;
    R.op1 = (float)((1.0 / 9.0) * gp);
    R.op5 = (float)((1.0 / 36.0) * gp);
  }
  if (wrap_m) {
    const double gm = (src_m - rd - 1.0) * invd;
    R.om1 = (float)((1.0 / 9.0) * gm);
    R.om5 = (float)((1.0 / 36.0) * gm);
  }
  const float r = (float)rd;
  const float inv = (float)invd;
  R.r = r;
  R.inv_r = inv;
  R.lr0b = 0.5f * (1.0f + D.c_tau * inv * inv);
  R.hcs2r = (float)(0.5 / 3.0) * inv;
  R.ar0 = inv * (float)(1.0 / 3.0);
  R.ar1 = 2.0f * D.c_tau * inv * inv;
  R.omT1 = D.omc * (1.0f + D.tau_T * inv);
  R.omT3 = D.omc * (1.0f - D.tau_T * inv);
  return R;
}

// Columns 0 and nz-1 are boundary nodes: no-slip walls, or inlet and outlet.
__host__ __device__ inline bool z_bounded(const InstDev& D) {
  return D.side_z == SIDE_WALL || D.side_z == SIDE_FLOW;
}

__host__ __device__ inline bool is_boundary(const InstDev& D, int j, int k) {
  return (D.side_rmin == SIDE_WALL && j == 0) || (D.side_rmax == SIDE_WALL && j == D.nr - 1) ||
         (z_bounded(D) && (k == 0 || k == D.nz - 1));
}

// Radial wall nodes beside fluid rows can be computed in the step by their
// own lanes (wall_lane_inputs, step kernels with wall lanes), which load
// their owner's populations.  That is safe only in the owner's wave, where the
// loads precede the owner's in-place stores: always at r_min (columns 0 and
// 1), at r_max unless column nr - 1 starts a new wave; otherwise the owner
// computes the wall node (wall_node).
__host__ __device__ inline bool wall_lane_rmax(const InstDev& D) {
  return (D.nr - 1) % LANES_R != 0;
}

__host__ __device__ inline uint8_t node_mask(const InstDev& D, int j, int k) {
  uint8_t m = 0;
  if (D.side_rmin == SIDE_WALL && j == 0) m |= MASK_RMIN;
  if (D.side_rmax == SIDE_WALL && j == D.nr - 1) m |= MASK_RMAX;
  if (z_bounded(D) && k == 0) m |= MASK_ZMIN;
  if (z_bounded(D) && k == D.nz - 1) m |= MASK_ZMAX;
  if (D.side_rmin == SIDE_AXIS && j == 0) m |= MASK_AXIS;
  return m;
}

// Isoflux wall node (Sec. 4.4): true, with q = q'/k, when wall node (mask m,
// column k) lies in the heated window of a flux wall and no fixed-temperature
// wall meets there.
__host__ __device__ inline bool flux_node(const InstDev& D, uint8_t m, int k, float& q) {
  if ((m & MASK_RMIN) && D.therm_rmin == THERM_FIXED) return false;
  if ((m & MASK_RMAX) && D.therm_rmax == THERM_FIXED) return false;
  if ((m & (MASK_ZMIN | MASK_ZMAX)) && D.therm_z == THERM_FIXED) return false;
  if (k < D.qk_lo || k > D.qk_hi) return false;
  if ((m & MASK_RMIN) && D.therm_rmin == THERM_FLUX) {
    q = D.q_rmin;
    return true;
  }
  if ((m & MASK_RMAX) && D.therm_rmax == THERM_FLUX) {
    q = D.q_rmax;
    return true;
  }
  return false;
}

// Reciprocal and square root from gfx950's single instructions (v_rcp_f32,
// v_sqrt_f32, about 1 ulp) with one Newton correction each, rather than the
// correctly rounded sequences that '/' and sqrtf compile to (about ten
// instructions each, with scaling and special-case handling that the step's
// finite, normal operands never need): a node update takes six reciprocals
// and four square roots, and the 16-bit step is bound by its vector-ALU
// instructions.  Without the corrections the 1-ulp errors are biased and
// accumulate over a run (measured: 5e-5 in rho - 1 after 300 steps of the
// Sec. 4.3 annulus); with them the results stay within the FP32 parity bound.
// Host code (descriptors only) divides exactly.
__host__ __device__ inline float frcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(__builtin_fmaf(-x, r, 1.0f), r, r);  // r (2 - x r)
#else
  return 1.0f / x;
#endif
}
__host__ __device__ inline float fsqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float y = __builtin_amdgcn_sqrtf(x);
  const float h = 0.5f * __builtin_amdgcn_rcpf(y);  // y = 0 gives h = inf and a NaN below
  const float c = __builtin_fmaf(__builtin_fmaf(-y, y, x), h, y);  // y + (x - y^2) / (2 y)
  return y > 0.0f ? c : y;
#else
  return sqrtf(x);
#endif
}

// Porosity, phi nu / K and phi F_phi / sqrt(K) at a node (Eqs. 6, 8).
// From the porosity value of the node (phi_raw: the field value, or unused
// when the porosity is uniform).
__host__ __device__ inline void porosity_of(const InstDev& D, float phi_raw, float& phi, float& cD,
                                            float& cF) {
  if (D.phi_mode == 0) {
    phi = D.phiu;
    cD = D.cD;
    cF = D.cF;
  } else {
    phi = phi_raw;
    const float iph = frcp(phi);
    const float q = (1.0f - phi) * iph;
    cD = D.C1 * q * q;
    cF = D.phi_mode == 1 ? D.C2 * q * iph : D.C3 * (1.0f - phi) * frcp(fsqrt(phi));
  }
}
__host__ __device__ inline void porosity(const InstDev& D, int64_t o, float& phi, float& cD,
                                         float& cF) {
  if (D.phi_mode == 0) {
    phi = D.phiu;
    cD = D.cD;
    cF = D.cF;
  } else {
    phi = D.phi[o];
    const float iph = frcp(phi);
    const float q = (1.0f - phi) * iph;
    cD = D.C1 * q * q;
    cF = D.phi_mode == 1 ? D.C2 * q * iph : D.C3 * (1.0f - phi) * frcp(fsqrt(phi));
  }
}

// delta += M^{-1} X for moment increments X_1..X_8 (X_0 = 0); M^{-1} = M^T
// diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4), M of Eq. (18).
__host__ __device__ inline void back_transform(float d[9], float X1, float X2, float X3, float X4,
                                               float X5, float X6, float X7, float X8) {
  const float a1 = X1 * (float)(1.0 / 36.0), a2 = X2 * (float)(1.0 / 36.0);
  const float a3 = X3 * (float)(1.0 / 6.0), a4 = X4 * (float)(1.0 / 12.0);
  const float a5 = X5 * (float)(1.0 / 6.0), a6 = X6 * (float)(1.0 / 12.0);
  const float a7 = X7 * 0.25f, a8 = X8 * 0.25f;
  const float e = -a1 - 2.0f * a2;      // common part of directions 1-4
  const float c = 2.0f * a1 + a2;       // common part of directions 5-8
  const float pr = a3 + a4, pz = a5 + a6;
  d[0] += -4.0f * a1 + 4.0f * a2;
  d[1] += e + a3 - 2.0f * a4 + a7;
  d[2] += e + a5 - 2.0f * a6 - a7;
  d[3] += e - a3 + 2.0f * a4 + a7;
  d[4] += e - a5 + 2.0f * a6 - a7;
  d[5] += c + pr + pz + a8;
  d[6] += c - pr + pz - a8;
  d[7] += c - pr - pz + a8;
  d[8] += c + pr - pz - a8;
}

// Moment-space source S / r of Eq. (24) with F~ = (F_r + a_r, F_z) (Eq. 25);
// unless printed, the a_r part is not divided by phi (see the header).
__host__ __device__ inline void source(bool printed, float rho, float ur, float uz, float iphi,
                                       float Fr, float Fz, float ar, float& S1, float& S7,
                                       float& S8) {
  if (printed) {
    const float Ftr = Fr + ar;
    S1 = 6.0f * rho * (ur * Ftr + uz * Fz) * iphi;
    S7 = 2.0f * rho * (ur * Ftr - uz * Fz) * iphi;
    S8 = rho * (ur * Fz + uz * Ftr) * iphi;
  } else {
    S1 = 6.0f * rho * ((ur * Fr + uz * Fz) * iphi + ur * ar);
    S7 = 2.0f * rho * ((ur * Fr - uz * Fz) * iphi + ur * ar);
    S8 = rho * ((ur * Fz + uz * Fr) * iphi + uz * ar);
  }
}

__host__ __device__ inline bool fluid_dest(const InstDev& D, int j, int& k) {
  if (j < 0 || j >= D.nr) return false;
  if (D.side_z == SIDE_PERIODIC) {
    if (k < 0) k += D.nz;
    if (k >= D.nz) k -= D.nz;
  } else if (k < 0 || k >= D.nz) {
    return false;
  }
  return !is_boundary(D, j, k);
}

// Fluid-node state kept for the wall nodes a thread owns.
struct NodeState {
  float drho, rho, ur, uz, theta, T;
  float n1, n2, n3, n4, n5, n6, n7, n8;  // non-equilibrium moments / r
  float t[5];                            // stored temperature slots
};

template <typename S, bool ODD, typename A>
__host__ __device__ inline void store_wall(const InstDev& D, const A& P, int jb, int kb, const float d[9],
                                           const float tg[5], Dither& rn) {
  constexpr int EXr[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  constexpr int EZr[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  constexpr int MIR[9] = {0, 3, 2, 1, 4, 6, 5, 8, 7};  // e_r reversed
  // A population that leaves row 0 towards an axis lands in the mirror row,
  // whose slot i is slot i* of row 0: the boundary nodes of row 0 feed the
  // fluid nodes of row 0 through it.
  for (int i = 1; i < 9; ++i) {
    int jd = jb + EXr[i], kd = kb + EZr[i], slot = i;
    if (jd < 0 && D.side_rmin == SIDE_AXIS) {
      jd = 0;
      slot = MIR[i];
    }
    if (!fluid_dest(D, jd, kd)) continue;
    if (ODD)
      P.st(slot, row_off(kd, D.stride) + jd, d[i], rn.next());
    else
      P.st(OPP[i], row_off(kb, D.stride) + jb, d[i], rn.next());
  }
  for (int i = 1; i < 5; ++i) {
    int jd = jb + EXr[i], kd = kb + EZr[i], slot = i;
    if (jd < 0 && D.side_rmin == SIDE_AXIS) {
      jd = 0;
      slot = MIR[i];
    }
    if (!fluid_dest(D, jd, kd)) continue;
    if (ODD)
      P.st(9 + slot, row_off(kd, D.stride) + jd, tg[i], rn.next());
    else
      P.st(9 + OPP[i], row_off(kb, D.stride) + jb, tg[i], rn.next());
  }
}

// Boundary node b = x + (dr, dz) owned by fluid node x (non-equilibrium
// extrapolation, Sec. 4) with its own macroscopic state: no-slip walls take
// rho_B, u = 0 and the wall temperature; with inlet/outlet columns (Sec. 4.1)
// the inlet takes rho_B, u = (0, u_in) and the inlet temperature, the outlet
// rho = 1 and B's u and T.  Radial walls win at corners.
template <typename S, bool ODD, int MODE, typename A>
__host__ __device__ inline void wall_node(const InstDev& D, const A& P, const NodeState& B, float rB,
                                          int j, int k, int dr, int dz, int mac_slot,
                                          const FieldOut& fo, Dither& rn) {
  const int jb = j + dr, kb = k + dz;
  const float rb = rB + (float)dr;
  const float inv_rb = frcp(rb);
  const int64_t ob = row_off(kb, D.stride) + jb;
  float phib, cDb, cFb;
  porosity_of(D, D.phi_mode == 0 ? 0.0f : D.phi[ob], phib, cDb, cFb);
  const uint8_t m = node_mask(D, jb, kb);
  float drho = B.drho, urb = 0.0f, uzb = 0.0f;
  const bool moving = D.side_z == SIDE_FLOW && !(m & (MASK_RMIN | MASK_RMAX));  // inlet or outlet
  if (moving) {
    if (m & MASK_ZMIN) {
      uzb = D.u_in;
    } else {
      drho = 0.0f;  // outlet: rho = rho_0 = 1
      urb = B.ur;
      uzb = B.uz;
    }
  }
  const float rhob = 1.0f + drho;
  float Tb = B.T;
  if ((m & MASK_RMIN) && D.therm_rmin == THERM_FIXED) Tb = D.T_rmin;
  else if ((m & MASK_RMAX) && D.therm_rmax == THERM_FIXED) Tb = D.T_rmax;
  else if ((m & MASK_ZMIN) && D.therm_z == THERM_FIXED) Tb = D.T_zmin;
  else if ((m & MASK_ZMAX) && D.therm_z == THERM_FIXED && D.side_z != SIDE_FLOW) Tb = D.T_zmax;
  else {
    // Isoflux: one-sided difference over the unit spacing to B gives -dT/dn = q'/k.
    float q;
    if (flux_node(D, m, kb, q)) Tb = B.T + q;
  }

  if (MODE != MODE_FIELDS) {
    // Flow: m+(b) = m^eq(b) + (I - L)(r_B / r_b) n(B) + (I - L/2) S(b), all / r_b,
    // as deviations from the quiescent post-collision moments
    // (1, -2, 1, c_s^2 / (2 r_b), -c_s^2 / (2 r_b), 0, 0, 0, 0).
    // Temperature: g+(b) = g^eq(T_b, u_b) + (1 - omega_i(r_b)) g^neq(B) + psi_i(b).
    // No-slip walls (u_b = 0) take a short path: the velocity terms vanish.
    // At one wave per SIMD (small grids) the wall work sits on the critical
    // path of the owner's wave, so it is kept as short as the case allows.
    const float q = rB * inv_rb;
    const float hb = 0.5f * CS2 * inv_rb;
    const float Gz = D.gbeta * (Tb - D.T_ref) + D.accel_z;
    const float eu[5] = {0.0f, B.ur, B.uz, -B.ur, -B.uz};
    const float wt[5] = {WT0, WT1, WT1, WT1, WT1};
    const float tb1 = D.tau_T * inv_rb;
    const float om[5] = {D.omc, D.omc * (1.0f + tb1), D.omc, D.omc * (1.0f - tb1), D.omc};
    float qn[5];
    for (int i = 1; i < 5; ++i) qn[i] = B.t[i] - wt[i] * B.theta;
    qn[0] = -((qn[1] + qn[3]) + (qn[2] + qn[4]));
    float d[9], tg[5];
    d[0] = W0 * drho;
    d[1] = d[2] = d[3] = d[4] = W1 * drho;
    d[5] = d[6] = d[7] = d[8] = W5 * drho;
    if (!moving) {
      const float S3 = rhob * (phib * D.accel_r + CS2 * inv_rb), S5 = rhob * phib * Gz;
      back_transform(d, (1.0f - D.s_e) * q * B.n1, (1.0f - D.s_eps) * q * B.n2,
                     (1.0f - D.s_j) * q * B.n3 + (1.0f - 0.5f * D.s_j) * S3 - hb,
                     (1.0f - D.s_q) * q * B.n4 - (1.0f - 0.5f * D.s_q) * S3 + hb,
                     (1.0f - D.s_j) * q * B.n5 + (1.0f - 0.5f * D.s_j) * S5,
                     (1.0f - D.s_q) * q * B.n6 - (1.0f - 0.5f * D.s_q) * S5,
                     (1.0f - D.s_nu) * q * B.n7, (1.0f - D.s_nu) * q * B.n8);
      for (int i = 0; i < 5; ++i) {
        const float gneq = qn[i] - 5.0f * wt[i] * B.T * eu[i];
        tg[i] = wt[i] * (Tb - D.T_s) + (1.0f - om[i]) * gneq;
      }
    } else {
      const float iphib = frcp(phib);
      const float drag = cDb + cFb * fsqrt(urb * urb + uzb * uzb);
      const float Frb = phib * D.accel_r - drag * urb, Fzb = phib * Gz - drag * uzb;
      const float arb = CS2 * inv_rb - 2.0f * D.c_tau * urb * inv_rb * inv_rb;  // Eq. (25)
      float S1, S7, S8;
      source(D.src_printed != 0, rhob, urb, uzb, iphib, Frb, Fzb, arb, S1, S7, S8);
      const float S3 = rhob * (Frb + arb), S5 = rhob * Fzb;
      const float ru2 = 3.0f * rhob * (urb * urb + uzb * uzb) * iphib;
      back_transform(d, ru2 + (1.0f - D.s_e) * q * B.n1 + (1.0f - 0.5f * D.s_e) * S1,
                     -ru2 + (1.0f - D.s_eps) * q * B.n2 - (1.0f - 0.5f * D.s_eps) * S1,
                     rhob * urb + (1.0f - D.s_j) * q * B.n3 + (1.0f - 0.5f * D.s_j) * S3 - hb,
                     -rhob * urb + (1.0f - D.s_q) * q * B.n4 - (1.0f - 0.5f * D.s_q) * S3 + hb,
                     rhob * uzb + (1.0f - D.s_j) * q * B.n5 + (1.0f - 0.5f * D.s_j) * S5,
                     -rhob * uzb + (1.0f - D.s_q) * q * B.n6 - (1.0f - 0.5f * D.s_q) * S5,
                     rhob * (urb * urb - uzb * uzb) * iphib + (1.0f - D.s_nu) * q * B.n7 +
                         (1.0f - 0.5f * D.s_nu) * S7,
                     rhob * urb * uzb * iphib + (1.0f - D.s_nu) * q * B.n8 +
                         (1.0f - 0.5f * D.s_nu) * S8);
      const float eb[5] = {0.0f, urb, uzb, -urb, -uzb};
      const float psib = -urb * inv_rb;
      for (int i = 0; i < 5; ++i) {
        const float gneq = qn[i] - 5.0f * wt[i] * B.T * eu[i];
        const float geqm = wt[i] * Tb * 5.0f * eb[i];  // velocity part of g^eq(T_b, u_b)
        tg[i] = wt[i] * (Tb - D.T_s) + geqm + (1.0f - om[i]) * gneq + psib * (wt[i] * Tb + geqm);
      }
    }
    store_wall<S, ODD>(D, P, jb, kb, d, tg, rn);
  }
  if (MODE == MODE_STEP_MACRO) {
    float* mac = mac_slot ? D.mac[1] : D.mac[0];  // select, not index: keeps D out of scratch
    mac[ob] = uzb;
    mac[D.plane + ob] = urb;
    mac[2 * D.plane + ob] = Tb;
  }
  if (MODE == MODE_FIELDS) {
    const int64_t o = (int64_t)kb * D.nr + jb;
    if (fo.uz) fo.uz[o] = uzb;
    if (fo.ur) fo.ur[o] = urb;
    if (fo.p) fo.p[o] = rhob * CS2 / phib;
    if (fo.T) fo.T[o] = Tb;
    if (fo.mask) fo.mask[o] = m;
    if (fo.drho) fo.drho[o] = drho;
  }
}

// The populations arriving at fluid node (j, k) (as stored, unscaled to
// FP32) and its porosity value.  Each slot is read and written by one node
// only in a step, so these loads may be issued before earlier nodes of the
// same thread are updated.
template <typename S, bool ODD, bool BUF = false>
__host__ __device__ inline void node_load(const InstDev& D, const RowC& R, int j, int k, float s[9],
                                          float t[5], float& phi_raw) {
  const PopAcc<S, BUF> P(D);
  const int st = D.stride;
  int km = k - 1, kp = k + 1;
  if (D.side_z == SIDE_PERIODIC) {
    if (km < 0) km += D.nz;
    if (kp >= D.nz) kp -= D.nz;
  }
  const int64_t rowm = row_off(km, st), row0 = row_off(k, st), rowp = row_off(kp, st);
  const int64_t o = row0 + j;
  if constexpr (sizeof(S) == 4) {
    if (!ODD) {
#pragma unroll
      for (int q = 0; q < 9; ++q) s[q] = P.ld(q, o);
      t[0] = D.g0[o];
#pragma unroll
      for (int q = 1; q < 5; ++q) t[q] = P.ld(9 + q, o);
    } else {
      const int64_t cm = R.cm, cp = R.cp;
      s[0] = P.ld(0, o);
      s[1] = P.ld(R.mir ? 1 : 3, row0 + cm);
      s[2] = P.ld(4, rowm + j);
      s[3] = P.ld(1, row0 + cp);
      s[4] = P.ld(2, rowp + j);
      s[5] = P.ld(R.mir ? 8 : 7, rowm + cm);
      s[6] = P.ld(8, rowm + cp);
      s[7] = P.ld(5, rowp + cp);
      s[8] = P.ld(R.mir ? 5 : 6, rowp + cm);
      t[0] = D.g0[o];
      t[1] = P.ld(R.mir ? 10 : 12, row0 + cm);
      t[2] = P.ld(13, rowm + j);
      t[3] = P.ld(10, row0 + cp);
      t[4] = P.ld(11, rowp + j);
    }
  } else {
    // 16-bit storage: f_i and g_i of the axial directions come in pairs
    if (!ODD) {
      s[0] = P.ld(0, o);
#pragma unroll
      for (int a = 0; a < 4; ++a) P.ld_pair(a, o, s[a + 1], t[a + 1]);
#pragma unroll
      for (int q = 5; q < 9; ++q) s[q] = P.ld(q, o);
      t[0] = D.g0[o];
    } else {
      const int64_t cm = R.cm, cp = R.cp;
      s[0] = P.ld(0, o);
      P.ld_pair(R.mir ? 0 : 2, row0 + cm, s[1], t[1]);
      P.ld_pair(3, rowm + j, s[2], t[2]);
      P.ld_pair(0, row0 + cp, s[3], t[3]);
      P.ld_pair(1, rowp + j, s[4], t[4]);
      s[5] = P.ld(R.mir ? 8 : 7, rowm + cm);
      s[6] = P.ld(8, rowm + cp);
      s[7] = P.ld(5, rowp + cp);
      s[8] = P.ld(R.mir ? 5 : 6, rowp + cm);
      t[0] = D.g0[o];
    }
  }
  phi_raw = D.phi_mode == 0 ? 0.0f : D.phi[o];
}

// Slots of the populations arriving at fluid node (j, k) in the AA layout of
// the step's parity, as node_load reads them: value v (0..8: f_0..f_8,
// 9..12: g_1..g_4) sits in slot q[v] of node offset off[v]; o is the node's
// own offset (g_0 plane, porosity).  The step writes its post-collision f_i
// into the slot it read f_opposite(i) from, so these are also the slots it
// writes.  Used by the streaming-ceiling probe, whose identity update (every
// value stored back where node_load found it) leaves the state unchanged only
// if this map is node_load's.
template <bool ODD>
__host__ __device__ inline void node_slots(const InstDev& D, const RowC& R, int j, int k, int q[13],
                                           int64_t off[13], int64_t& o) {
  const int st = D.stride;
  int km = k - 1, kp = k + 1;
  if (D.side_z == SIDE_PERIODIC) {
    if (km < 0) km += D.nz;
    if (kp >= D.nz) kp -= D.nz;
  }
  const int64_t rowm = row_off(km, st), row0 = row_off(k, st), rowp = row_off(kp, st);
  o = row0 + j;
  if (!ODD) {
#pragma unroll
    for (int v = 0; v < 9; ++v) q[v] = v, off[v] = o;
#pragma unroll
    for (int v = 9; v < 13; ++v) q[v] = v + 1, off[v] = o;
  } else {
    const int64_t cm = R.cm, cp = R.cp;
    q[0] = 0, off[0] = o;
    q[1] = R.mir ? 1 : 3, off[1] = row0 + cm;
    q[2] = 4, off[2] = rowm + j;
    q[3] = 1, off[3] = row0 + cp;
    q[4] = 2, off[4] = rowp + j;
    q[5] = R.mir ? 8 : 7, off[5] = rowm + cm;
    q[6] = 8, off[6] = rowm + cp;
    q[7] = 5, off[7] = rowp + cp;
    q[8] = R.mir ? 5 : 6, off[8] = rowp + cm;
    q[9] = R.mir ? 10 : 12, off[9] = row0 + cm;
    q[10] = 13, off[10] = rowm + j;
    q[11] = 10, off[11] = row0 + cp;
    q[12] = 11, off[12] = rowp + j;
  }
}

// Streaming-ceiling probe: the stores of fluid node (j, k) with the step's
// memory traffic and no arithmetic.  After the step's loads (node_load) each
// value goes back, as the step orders its stores (f_i^+ into the slot of
// f_opposite(i), then g; in 16-bit storage the axial f and g of a slot pair
// in one word), into the slot it came from, its bits XORed with key: key = 0
// leaves the state as it was, and the compiler cannot drop the stores.  The
// porosity value is folded into the g_0 store the same way.
template <typename S, bool ODD, bool BUF>
__device__ inline void pattern_store(const InstDev& D, const RowC& R, int j, int k, const float s[9],
                                     const float t[5], float ph, uint32_t key) {
  constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  const PopAcc<S, BUF> P(D);
  int q[13];
  int64_t off[13], o;
  node_slots<ODD>(D, R, j, k, q, off, o);
  auto x = [key](float v) { return __uint_as_float(__float_as_uint(v) ^ key); };
  if constexpr (sizeof(S) == 4) {
#pragma unroll
    for (int i = 0; i < 9; ++i) P.st(q[OPP[i]], off[OPP[i]], x(s[OPP[i]]), 0u);
    D.g0[o] = __uint_as_float(__float_as_uint(t[0]) ^ (key & __float_as_uint(ph)));
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const int b = i <= 2 ? i + 2 : i - 2;  // opposite of i in D2Q5
      P.st(q[8 + b], off[8 + b], x(t[b]), 0u);
    }
  } else {
    P.st(q[0], off[0], x(s[0]), 0u);
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const int b = OPP[i];  // f_b and g_b share the word of slot pair q[b] - 1
      P.st_pair(q[b] - 1, off[b], x(s[b]), x(t[b]), 0u, 0u);
    }
#pragma unroll
    for (int i = 5; i < 9; ++i) P.st(q[OPP[i]], off[OPP[i]], x(s[OPP[i]]), 0u);
    D.g0[o] = __uint_as_float(__float_as_uint(t[0]) ^ (key & __float_as_uint(ph)));
  }
}

// Inputs of a radial wall lane's collision (step kernels with wall lanes).
// The lane holds its owner B (column j, radius r_B) and turns the fluid
// collision into the no-slip wall node b = j - wl at r_b = r_B - wl (Sec. 4,
// non-equilibrium extrapolation): its post-collision state is
//   m+(b) = m^eq(rho_B, 0) + (I - L)(r_B / r_b) n(B) + (I - L/2) S(b),
// all / r_b, as deviations from the quiescent post-collision moments.  So
// the pre-collision d becomes the rest equilibrium w_i (rho_B - 1) and the
// moment increments X of the back-transform become (1 - s_i)(r_B / r_b) n_i
// plus the wall's source, with the quiescent parts -+ c_s^2 / (2 r_b) of the
// radial moments; the thermal population along e_r = wl becomes
//   g+(b) = wt (T_b - T_s) + (1 - omega(r_b)) g^neq(B).
// The node's stores then write the wall node's outgoing populations (e_r =
// wl: directions 1, 5, 8 or 3, 6, 7, and the D2Q5 one) to the slots its
// fluid neighbours read; its other populations go to the wall column's own
// slots, which no fluid node reads (node_update_loaded).
__host__ __device__ inline void wall_lane_inputs(const InstDev& D, const NodeState& B, const float t[5],
                                                 float rB, int wl, int k, int64_t ob, float d[9],
                                                 float X[8], float& ga, float& Tb) {
  const bool lo = wl > 0;
  const float fs = (float)wl;
  const float inv_rb = frcp(rB - fs);
  const float phib = D.phi_mode == 0 ? D.phiu : D.phi[ob];
  Tb = B.T;
  const int th = lo ? D.therm_rmin : D.therm_rmax;
  if (th == THERM_FIXED) Tb = lo ? D.T_rmin : D.T_rmax;
  else if (th == THERM_FLUX && k >= D.qk_lo && k <= D.qk_hi) Tb = B.T + (lo ? D.q_rmin : D.q_rmax);
  const float drho = B.drho, rhob = 1.0f + drho;
  const float q = rB * inv_rb;
  const float hb = 0.5f * CS2 * inv_rb;
  const float Gz = D.gbeta * (Tb - D.T_ref) + D.accel_z;
  const float S3 = rhob * (phib * D.accel_r + CS2 * inv_rb), S5 = rhob * phib * Gz;
  X[0] = (1.0f - D.s_e) * q * B.n1;
  X[1] = (1.0f - D.s_eps) * q * B.n2;
  X[2] = (1.0f - D.s_j) * q * B.n3 + (1.0f - 0.5f * D.s_j) * S3 - hb;
  X[3] = (1.0f - D.s_q) * q * B.n4 - (1.0f - 0.5f * D.s_q) * S3 + hb;
  X[4] = (1.0f - D.s_j) * q * B.n5 + (1.0f - 0.5f * D.s_j) * S5;
  X[5] = (1.0f - D.s_q) * q * B.n6 - (1.0f - 0.5f * D.s_q) * S5;
  X[6] = (1.0f - D.s_nu) * q * B.n7;
  X[7] = (1.0f - D.s_nu) * q * B.n8;
  d[0] = W0 * drho;
#pragma unroll
  for (int i = 1; i < 5; ++i) d[i] = W1 * drho;
#pragma unroll
  for (int i = 5; i < 9; ++i) d[i] = W5 * drho;
  const float om = D.omc * (1.0f + fs * D.tau_T * inv_rb);
  const float tB = lo ? t[1] : t[3];
  ga = WT1 * (Tb - D.T_s) + (1.0f - om) * (tB - WT1 * B.theta - 5.0f * WT1 * B.T * fs * B.ur);
}

// Whether the predicate holds on any lane of the wave (on the host, for this
// node): a branch on it is taken by whole waves, so what follows stays one
// path for all lanes.
__host__ __device__ inline bool any_lane(bool p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __any(p);
#else
  return p;
#endif
}

// One fluid node (j, k) at one time step, from its loaded populations s, t
// and porosity value.  seed: random bits of this step for stochastic
// rounding of 16-bit storage.
template <typename S, bool ODD, int MODE, bool BUF = false, bool WL = false>
__host__ __device__ inline void node_update_loaded(const InstDev& D, const RowC& R, int j, int k,
                                                   int mac_slot, const FieldOut& fo, uint32_t seed,
                                                   const float s[9], const float t_in[5],
                                                   float phi_raw, int wl = 0) {
  const PopAcc<S, BUF> P(D);
  const int64_t pl = D.plane;
  const int st = D.stride;
  int km = k - 1, kp = k + 1;
  if (D.side_z == SIDE_PERIODIC) {
    if (km < 0) km += D.nz;
    if (kp >= D.nz) kp -= D.nz;
  }
  const int64_t rowm = row_off(km, st), row0 = row_off(k, st), rowp = row_off(kp, st);
  const int64_t o = row0 + j;
  Dither rn(mix32(seed ^ (uint32_t)(o - wl)));  // a wall lane draws its wall node's stream
  float t[5] = {t_in[0], t_in[1], t_in[2], t_in[3], t_in[4]};
  float phi, cD, cF;
  porosity_of(D, phi_raw, phi, cD, cF);

  // Rescale to this node's frame: d_i = fhat_i - w_i (1 - e_ir / (2 r)).
  float d[9];
  d[0] = s[0];
  d[2] = s[2];
  d[4] = s[4];
  d[1] = s[1] * R.rp + R.op1;
  d[5] = s[5] * R.rp + R.op5;
  d[8] = s[8] * R.rp + R.op5;
  d[3] = s[3] * R.rm + R.om1;
  d[6] = s[6] * R.rm + R.om5;
  d[7] = s[7] * R.rm + R.om5;

  // ---- macroscopic values ------------------------------------------------
  NodeState B;
  const float sa = d[1] + d[2] + d[3] + d[4], sd = d[5] + d[6] + d[7] + d[8];
  B.drho = d[0] + sa + sd;                                  // rho - 1, Eq. (26)
  B.rho = 1.0f + B.drho;
  const float inv_rho = frcp(B.rho);
  // sum e_r f / r = Jr - c_s^2 / (2 r); sum e_z f / r = Jz
  const float Jr = d[1] - d[3] + d[5] - d[6] - d[7] + d[8];
  const float Jz = d[2] - d[4] + d[5] + d[6] - d[7] - d[8];
  B.theta = t[0] + t[1] + t[2] + t[3] + t[4];               // T - T_s, Eq. (38)
  B.T = D.T_s + B.theta;
  const float Gr = D.accel_r;
  const float Gz = D.gbeta * B.theta + D.az_s;              // Eq. (7)
  const float vr = (Jr + R.hcs2r * B.drho) * inv_rho + 0.5f * phi * Gr;  // Eq. (29) / r
  const float vz = Jz * inv_rho + 0.5f * phi * Gz;
  const float lr0 = R.lr0b + 0.25f * cD;                    // Eq. (30) / r
  const float lz0 = 0.5f + 0.25f * cD;
  const float l1 = 0.5f * cF;
  const float vm = fsqrt(vr * vr + vz * vz);
  B.ur = vr * frcp(lr0 + fsqrt(lr0 * lr0 + l1 * vm));       // Eq. (28)
  B.uz = vz * frcp(lz0 + fsqrt(lz0 * lz0 + l1 * vm));
  const float ur = B.ur, uz = B.uz, rho = B.rho;

  if (MODE == MODE_STEP_MACRO) {
    float* mac = mac_slot ? D.mac[1] : D.mac[0];  // select, not index: keeps D out of scratch
    mac[o] = uz;
    mac[pl + o] = ur;
    mac[2 * pl + o] = B.T;
  }
  if (MODE == MODE_FIELDS) {
    const int64_t oo = (int64_t)k * D.nr + j;
    if (fo.uz) fo.uz[oo] = uz;
    if (fo.ur) fo.ur[oo] = ur;
    if (fo.p) fo.p[oo] = rho * CS2 / phi;
    if (fo.T) fo.T[oo] = B.T;
    if (fo.mask) fo.mask[oo] = node_mask(D, j, k);
    if (fo.drho) fo.drho[oo] = B.drho;
  }

  // ---- forces (Eq. 6) and the axisymmetric correction (Eq. 25) -----------
  const float um = fsqrt(ur * ur + uz * uz);
  const float drag = cD + cF * um;
  const float Fr = phi * Gr - drag * ur;
  const float Fz = phi * Gz - drag * uz;
  const float ar = R.ar0 - R.ar1 * ur;

  // ---- moments of d and the non-equilibrium part (Eqs. 16-20) -----------
  const float iphi = frcp(phi);
  const float ru2 = rho * (ur * ur + uz * uz) * iphi;
  B.n1 = (-4.0f * d[0] - sa + 2.0f * sd) + 2.0f * B.drho - 3.0f * ru2;
  B.n2 = (4.0f * d[0] - 2.0f * sa + sd) - B.drho + 3.0f * ru2;
  const float m4 = -2.0f * d[1] + 2.0f * d[3] + d[5] - d[6] - d[7] + d[8];
  B.n3 = (Jr - R.hcs2r) - rho * ur;
  B.n4 = (m4 + R.hcs2r) + rho * ur;
  B.n5 = Jz - rho * uz;
  B.n6 = (-2.0f * d[2] + 2.0f * d[4] + d[5] + d[6] - d[7] - d[8]) + rho * uz;
  B.n7 = (d[1] - d[2] + d[3] - d[4]) - rho * (ur * ur - uz * uz) * iphi;
  B.n8 = (d[5] - d[6] + d[7] - d[8]) - rho * ur * uz * iphi;

  // Where the stores go: the node's own position and neighbour columns, or
  // for a radial wall lane (WL kernels, wl = +-1, node (j, k) being its
  // owner) its wall node jb = j - wl, whose missing neighbour column is the
  // wall column itself (see wall_lane_inputs).
  int js = j, cms = R.cm, cps = R.cp;
  int64_t os = o;
  if (MODE != MODE_FIELDS) {
    // ---- source (Eq. 24) and relaxation (Eq. 21) --------------------------
    float S1, S7, S8;
    source(D.src_printed != 0, rho, ur, uz, iphi, Fr, Fz, ar, S1, S7, S8);
    const float S5 = rho * Fz;
    // The radial-momentum and radial-flux increments are written so that the
    // quiescent parts (c_s^2 / (2 r) in n_3, n_4 and c_s^2 / r in S_3) and
    // the change of reference state (-c_s^2 / r in moment 3, +c_s^2 / r in
    // moment 4) cancel exactly: what remains scales with rho - 1 and u.
    const float S3d = rho * (Fr - R.ar1 * ur);  // S_3 minus its quiescent part rho c_s^2 / r
    const float X3 = -D.s_j * (Jr - rho * ur) + (1.0f - 0.5f * D.s_j) * S3d +
                     (2.0f - D.s_j) * R.hcs2r * B.drho;
    const float X4 = -D.s_q * (m4 + rho * ur) - (1.0f - 0.5f * D.s_q) * S3d -
                     (2.0f - D.s_q) * R.hcs2r * B.drho;
    float X[8] = {-D.s_e * B.n1 + (1.0f - 0.5f * D.s_e) * S1,
                  -D.s_eps * B.n2 - (1.0f - 0.5f * D.s_eps) * S1,
                  X3,
                  X4,
                  -D.s_j * B.n5 + (1.0f - 0.5f * D.s_j) * S5,
                  -D.s_q * B.n6 - (1.0f - 0.5f * D.s_q) * S5,
                  -D.s_nu * B.n7 + (1.0f - 0.5f * D.s_nu) * S7,
                  -D.s_nu * B.n8 + (1.0f - 0.5f * D.s_nu) * S8};

    // ---- temperature collision (Eqs. 33-37) ------------------------------
    // q_i = g_i - wt_i T is the part of g - g^eq that does not depend on u;
    // q_0 is formed as -(q_1 + ... + q_4) so that the rounding of theta and of
    // the FP32 weights cannot leak into sum_i g_i step after step.
    const float Tn = B.T;
    const float wT0 = WT0 * Tn, wT1 = WT1 * Tn;
    const float psi = -ur * R.inv_r;
    float tg[5];
    {
      const float e1 = 5.0f * ur, e2 = 5.0f * uz;
      const float q1 = t[1] - WT1 * B.theta, q2 = t[2] - WT1 * B.theta;
      const float q3 = t[3] - WT1 * B.theta, q4 = t[4] - WT1 * B.theta;
      const float q0 = -((q1 + q3) + (q2 + q4));
      tg[0] = t[0] - D.omc * q0 + psi * wT0;
      tg[1] = t[1] - R.omT1 * (q1 - wT1 * e1) + psi * wT1 * (1.0f + e1);
      tg[2] = t[2] - D.omc * (q2 - wT1 * e2) + psi * wT1 * (1.0f + e2);
      tg[3] = t[3] - R.omT3 * (q3 + wT1 * e1) + psi * wT1 * (1.0f - e1);
      tg[4] = t[4] - D.omc * (q4 + wT1 * e2) + psi * wT1 * (1.0f - e2);
    }
    for (int q = 0; q < 5; ++q) B.t[q] = t[q];

    if constexpr (WL) {
      // A wave with a wall lane forms the wall node's inputs on every lane and
      // the wall lane selects them (per-lane selects, not a divergent branch,
      // so the back-transform and the stores below stay one path).
      if (any_lane(wl != 0)) {
        const bool isw = wl != 0;
        const int jw = j - wl;  // the wall column (the node's own column on fluid lanes)
        float dw[9], Xw[8], ga, Tb;
        // In the 16-bit kernels (four waves per SIMD, so 128 VGPRs) the wall
        // lane's radius and side pass through an empty asm statement: the
        // compiler then forms the wall inputs' per-lane products in every
        // node update of a wave with a wall lane, instead of hoisting them out
        // of the node loop and spilling them to scratch. Same operations.
        float rw = R.r;
        int wlw = wl;
#if defined(__HIP_DEVICE_COMPILE__)
        if constexpr (sizeof(S) == 2) asm volatile("" : "+v"(rw), "+v"(wlw));
#endif
        wall_lane_inputs(D, B, t, rw, wlw, k, row0 + jw, dw, Xw, ga, Tb);
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = isw ? dw[i] : d[i];
#pragma unroll
        for (int i = 0; i < 8; ++i) X[i] = isw ? Xw[i] : X[i];
        tg[1] = wl > 0 ? ga : tg[1];
        tg[3] = wl < 0 ? ga : tg[3];
        js = jw;
        os = row0 + jw;
        cms = wl > 0 ? jw : (wl < 0 ? jw - 1 : cms);  // the missing neighbour column is the wall column itself
        cps = wl < 0 ? jw : (wl > 0 ? jw + 1 : cps);
        if (MODE == MODE_STEP_MACRO && isw) {
          float* mac = mac_slot ? D.mac[1] : D.mac[0];
          mac[os] = 0.0f;
          mac[pl + os] = 0.0f;
          mac[2 * pl + os] = Tb;
        }
      }
    }

    // ---- back-transform (Eq. 22) ------------------------------------------
    back_transform(d, X[0], X[1], X[2], X[3], X[4], X[5], X[6], X[7]);

    // ---- stream and store --------------------------------------------------
    if constexpr (sizeof(S) == 4) {
      if (!ODD) {
        P.st(0, os, d[0], rn.next());
        P.st(3, os, d[1], rn.next());
        P.st(4, os, d[2], rn.next());
        P.st(1, os, d[3], rn.next());
        P.st(2, os, d[4], rn.next());
        P.st(7, os, d[5], rn.next());
        P.st(8, os, d[6], rn.next());
        P.st(5, os, d[7], rn.next());
        P.st(6, os, d[8], rn.next());
        D.g0[os] = tg[0];
        P.st(12, os, tg[1], rn.next());
        P.st(13, os, tg[2], rn.next());
        P.st(10, os, tg[3], rn.next());
        P.st(11, os, tg[4], rn.next());
      } else {
        const int64_t cm = cms, cp = cps;
        P.st(0, os, d[0], rn.next());
        P.st(1, row0 + cp, d[1], rn.next());
        P.st(2, rowp + js, d[2], rn.next());
        P.st(R.mir ? 1 : 3, row0 + cm, d[3], rn.next());
        P.st(4, rowm + js, d[4], rn.next());
        P.st(5, rowp + cp, d[5], rn.next());
        P.st(R.mir ? 5 : 6, rowp + cm, d[6], rn.next());
        P.st(R.mir ? 8 : 7, rowm + cm, d[7], rn.next());
        P.st(8, rowm + cp, d[8], rn.next());
        D.g0[os] = tg[0];
        P.st(10, row0 + cp, tg[1], rn.next());
        P.st(11, rowp + js, tg[2], rn.next());
        P.st(R.mir ? 10 : 12, row0 + cm, tg[3], rn.next());
        P.st(13, rowm + js, tg[4], rn.next());
      }
    } else {
      // 16-bit storage: f_i^+ and g_i^+ of each axial direction land in the
      // two halves of one word (slots q and q + 9 of one node)
      uint32_t r[13];
#pragma unroll
      for (int i = 0; i < 13; ++i) r[i] = rn.next();
      if (!ODD) {
        P.st(0, os, d[0], r[0]);
        P.st_pair(2, os, d[1], tg[1], r[1], r[9]);   // slots 3, 12
        P.st_pair(3, os, d[2], tg[2], r[2], r[10]);  // slots 4, 13
        P.st_pair(0, os, d[3], tg[3], r[3], r[11]);  // slots 1, 10
        P.st_pair(1, os, d[4], tg[4], r[4], r[12]);  // slots 2, 11
        P.st(7, os, d[5], r[5]);
        P.st(8, os, d[6], r[6]);
        P.st(5, os, d[7], r[7]);
        P.st(6, os, d[8], r[8]);
      } else {
        const int64_t cm = cms, cp = cps;
        P.st(0, os, d[0], r[0]);
        P.st_pair(0, row0 + cp, d[1], tg[1], r[1], r[9]);
        P.st_pair(1, rowp + js, d[2], tg[2], r[2], r[10]);
        P.st_pair(R.mir ? 0 : 2, row0 + cm, d[3], tg[3], r[3], r[11]);
        P.st_pair(3, rowm + js, d[4], tg[4], r[4], r[12]);
        P.st(5, rowp + cp, d[5], r[5]);
        P.st(R.mir ? 5 : 6, rowp + cm, d[6], r[6]);
        P.st(R.mir ? 8 : 7, rowm + cm, d[7], r[7]);
        P.st(8, rowm + cp, d[8], r[8]);
      }
      D.g0[os] = tg[0];
    }
  } else {
    for (int q = 0; q < 5; ++q) B.t[q] = t[q];
  }

  // ---- wall nodes owned by this node ---------------------------------------
  // (after the fluid node's stores: only B stays live across them)
  if constexpr (WL && MODE != MODE_FIELDS) {
    if (wl != 0) return;  // a wall lane's wall node is stored above
  }
  const bool own_rm = D.side_rmin == SIDE_WALL && j == 1;
  const bool own_rp = D.side_rmax == SIDE_WALL && j == D.nr - 2;
  const bool own_zm = z_bounded(D) && k == 1;
  const bool own_zp = z_bounded(D) && k == D.nz - 2;
  // In the step kernels with wall lanes the radial wall nodes beside fluid
  // rows are their own lanes' (wall_lane_inputs, where wall_lane_rmax allows);
  // owners keep the rest: the z-wall nodes and the corners.
  const bool rad_m = MODE == MODE_FIELDS || !WL;
  const bool rad_p = MODE == MODE_FIELDS || !WL || !wall_lane_rmax(D);
  // Each (dr, dz) below is a separate inlined copy with constant offsets: on
  // annuli, where corner owners take three wall nodes, these specialised
  // passes run faster than one generic pass walked per lane.
  // Where LBM_OWNER_WALLS_UNLIKELY is defined (the file of the 16-bit
  // kernels) the branch is marked unlikely, which keeps the compiler from
  // hoisting parts of the wall-node work into every fluid node's update.
  const bool owns = (rad_m && own_rm) || (rad_p && own_rp) || own_zm || own_zp;
#if defined(LBM_OWNER_WALLS_UNLIKELY)
  if (__builtin_expect(owns, 0)) {
#else
  if (owns) {
#endif
    for (int dr = -1; dr <= 1; ++dr) {
      if ((dr == -1 && !own_rm) || (dr == 1 && !own_rp)) continue;
      for (int dz = -1; dz <= 1; ++dz) {
        if (dr == 0 && dz == 0) continue;
        if (dz == 0 && ((dr == -1 && !rad_m) || (dr == 1 && !rad_p))) continue;
        if ((dz == -1 && !own_zm) || (dz == 1 && !own_zp)) continue;
        wall_node<S, ODD, MODE>(D, P, B, R.r, j, k, dr, dz, mac_slot, fo, rn);
      }
    }
  }
}

// One fluid node (j, k) at one time step (load, then update).
template <typename S, bool ODD, int MODE, bool BUF = false, bool WL = false>
__host__ __device__ inline void node_update(const InstDev& D, const RowC& R, int j, int k,
                                            int mac_slot, const FieldOut& fo, uint32_t seed,
                                            int wl = 0) {
  float s[9], t[5], ph;
  node_load<S, ODD, BUF>(D, R, j, k, s, t, ph);
  node_update_loaded<S, ODD, MODE, BUF, WL>(D, R, j, k, mac_slot, fo, seed, s, t, ph, wl);
}

// Start state of node (j, k) (reading: f = f^eq - S~/2, g = g^eq), written
// in the even-time layout with every slot in its source's frame.
template <typename S>
__host__ __device__ inline void init_node(const InstDev& D, int j, int k, float uz, float ur,
                                          float T) {
  constexpr int EXr[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  constexpr int EZr[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  S* P = (S*)D.pop;
  const int64_t o = (int64_t)k * D.stride + j;
  const double r = (double)D.r0 + j;
  float phi, cD, cF;
  porosity(D, o, phi, cD, cF);
  const float iphi = 1.0f / phi;
  const float inv_r = (float)(1.0 / r);
  const float theta = T - D.T_ref;
  const float Gz = D.gbeta * theta + D.accel_z;
  const float um = sqrtf(ur * ur + uz * uz);
  const float Fr = phi * D.accel_r - (cD + cF * um) * ur;
  const float Fz = phi * Gz - (cD + cF * um) * uz;
  const float ar = CS2 * (1.0f - 2.0f * D.c_tau * 3.0f * ur * inv_r) * inv_r;
  float S1, S7, S8;
  source(D.src_printed != 0, 1.0f, ur, uz, iphi, Fr, Fz, ar, S1, S7, S8);
  const float S3d = Fr - 2.0f * D.c_tau * ur * inv_r * inv_r;  // S_3 - c_s^2 / r at rho = 1
  const float S5 = Fz;
  const float u2 = (ur * ur + uz * uz) * iphi;
  // (m^eq - S/2) / r at rho = 1 minus the moments of the pre-collision
  // quiescent state (1, -2, 1, -c_s^2 / (2r), c_s^2 / (2r), 0, 0, 0, 0)
  float d[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  back_transform(d, 3.0f * u2 - 0.5f * S1, -3.0f * u2 + 0.5f * S1, ur - 0.5f * S3d,
                 -ur + 0.5f * S3d, uz - 0.5f * S5, -uz + 0.5f * S5,
                 (ur * ur - uz * uz) * iphi - 0.5f * S7, ur * uz * iphi - 0.5f * S8);
  const float w[9] = {W0, W1, W1, W1, W1, W5, W5, W5, W5};
  for (int i = 0; i < 9; ++i) {
    const int js = j - EXr[i];
    int ks = k - EZr[i];
    double rs = r - EXr[i];
    bool inside = true;
    if (js < 0) {
      if (D.side_rmin == SIDE_PERIODIC) rs = (double)D.r0 + D.nr - 1;
      else inside = D.side_rmin == SIDE_AXIS;
    }
    if (js >= D.nr) {
      if (D.side_rmax == SIDE_PERIODIC) rs = (double)D.r0;
      else inside = false;
    }
    if (D.side_z != SIDE_PERIODIC && (ks < 0 || ks >= D.nz)) inside = false;
    // stored in the source frame: s = (d - w (r_src - r + e) / r) r / r_src
    float v = d[i];
    if (inside && EXr[i] != 0)
      v = (float)(((double)d[i] - (double)w[i] * (rs - r + EXr[i]) / r) * (r / rs));
    Store<S>::st(P, slot_elem<S>(i, o, D.plane), v, D.st_scale);
  }
  const float eu[5] = {0.0f, ur, uz, -ur, -uz};
  const float wt[5] = {WT0, WT1, WT1, WT1, WT1};
  D.g0[o] = wt[0] * (T - D.T_s);
  for (int i = 1; i < 5; ++i)
    Store<S>::st(P, slot_elem<S>(9 + i, o, D.plane), wt[i] * (T * (1.0f + 5.0f * eu[i]) - D.T_s),
                 D.st_scale);
}

}  // namespace lbmaxi
