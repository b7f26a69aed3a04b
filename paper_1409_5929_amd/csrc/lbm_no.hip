// Warm-start network of the lattice Boltzmann solver: forward pass, loss,
// backward pass and Adam on gfx950 (layer definitions in include/lbm_no.h).
//
// Every convolution runs as GEMMs on MFMA (v_mfma_f32_16x16x32_bf16:
// bfloat16 operands, FP32 accumulation), with k = (cin, ky, kx) and p =
// (batch, y, x):
//   forward          z[o][p]  = sum_k W[o][k] col[k][p] + b[o] (im2col),
//                    for upsampling layers four phase GEMMs over the source
//                    grid (forward_up)
//   weight gradient  dW[o][k] = sum_p dz[o][p] col[k][p] (split over p),
//                    for upsampling layers over 2 x 2 box sums of dz (k_dmap)
//   input gradient   upsampling layers: a GEMM over the same box sums;
//                    stride-2 layers: four phase GEMMs over a shifted stack
//                    of dz (k_emap); 1 x 1 layers: one GEMM
// so no gradient is scattered back through an im2col (no col2im pass).
// Activations are kept channel-major, [C][batch][H][W], so each GEMM output
// is the next layer's input without a transpose.  Reductions (bias
// gradients, split partials, loss) run in a fixed order, so results do not
// depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lbm_no.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define NOCHK(call)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return fail(LBM_NO_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint16_t bf16_t;  // bfloat16 bit pattern

__host__ __device__ inline bf16_t to_bf16(float v) {  // round to nearest even (finite inputs)
  uint32_t u = __builtin_bit_cast(uint32_t, v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

constexpr int NT = 256;      // threads of a GEMM block (four waves)
constexpr int GBK = 64;      // k per LDS stage of the GEMM
constexpr int GLD = GBK + 8; // padded LDS row (bf16): 144 B, rows stay 16-byte aligned
constexpr int EW = 256;      // threads of the elementwise kernels

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// 8 bfloat16 of a row, row[k .. k + 7], zero at and beyond kend; one 16-byte
// load when vec (row and k 16-byte aligned) and the 8 lie before kend.
__device__ inline uint4 load8(const bf16_t* __restrict__ row, int k, int kend, bool vec) {
  if (vec && k + 8 <= kend) return *(const uint4*)(row + k);
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (k + i < kend) w[i >> 1] |= (uint32_t)row[k + i] << (16 * (i & 1));
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Halves h of the four words a, b (a in the low half): for the register
// transpose of the n-contiguous B operand.
__device__ inline uint32_t pick(uint32_t a, uint32_t b, int h) {
  return h ? (a >> 16) | (b & 0xFFFF0000u) : (a & 0xFFFFu) | (b << 16);
}
__device__ inline uint32_t word(const uint4& v, int d) { return d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w; }

// C[m][n] = sum_k A[m][k] B(k, n) (+ bias[m] in split 0) on bfloat16 operands
// with FP32 accumulation, on v_mfma_f32_16x16x32_bf16.
// A is k-contiguous (row m at A + m lda).  BKC: B(k, n) = B[n ldb + k];
// otherwise B(k, n) = B[k ldb + n].  Split z covers k in [z kchunk,
// (z + 1) kchunk) and writes C + z cz.
// Block: WM x (4 / WM) waves, each 64 x 64 outputs as 4 x 4 MFMA tiles of
// 16 x 16; k staged through LDS 64 at a time with k contiguous (B
// transposed on the way when n-contiguous: each thread turns a 4 (k) x 8 (n)
// block around in registers and writes eight 8-byte rows).  The next stage's
// operands are loaded into registers while the current one is multiplied.
// accumulate: C += instead of C =.  relu (single split): C = max(C, 0) as
// stored, the activation of a layer without a skip input.
// PH: four phase GEMMs of a stride-2 grid relation, phase q = (py, px) = (q
// / 2, q % 2), no split: A + ph.aoff[q], reduction length ph.K[q], B row k
// taken from row ph.base[q] + k (+ ph.gap[q] once k >= ph.run[q]), and column
// n = (b, y, x) of an Hn x Wn grid written to (b, 2y + py, 2x + px) of the
// 2Hn x 2Wn grid (row m of C at C + m ldc); bias in every phase.  PAIR:
// block z = py runs both px, each output pair one 8-byte store (C and its
// rows 8-byte aligned); otherwise block z = q runs one phase.
// vecA / vecB: rows 16-byte aligned (leading dimension a multiple of 8,
// aligned base, kchunk a multiple of 8), so whole 8-element chunks move as
// one 16-byte load; otherwise element by element.  Zero outside the
// matrices.
struct PhaseT {
  int64_t aoff[4];
  int K[4], base[4], run[4], gap[4];
  int Hn, Wn;
};
template <bool BKC, int WM, bool PH, bool PAIR>
__global__ __launch_bounds__(NT) void k_gemm(int M, int N, int K, const bf16_t* __restrict__ A,
                                             int64_t lda, int vecA, const bf16_t* __restrict__ B,
                                             int64_t ldb, int vecB, float* __restrict__ C, int64_t ldc,
                                             int64_t cz, int kchunk, const float* __restrict__ bias,
                                             int accumulate, PhaseT ph, int relu) {
  static_assert(!(PH && BKC) && (PH || !PAIR), "phase GEMMs take an n-contiguous B");
  constexpr int WN = 4 / WM, TBM = 64 * WM, TBN = 64 * WN;
  constexpr int NA = TBM * GBK / 8 / NT;   // 16-byte A chunks per thread and stage
  constexpr int NB = TBN * GBK / 8 / NT;   // 16-byte B chunks per thread and stage
  __shared__ __attribute__((aligned(16))) bf16_t As[TBM * GLD];
  __shared__ __attribute__((aligned(16))) bf16_t Bs[TBN * GLD];
  const int m0 = blockIdx.y * TBM, n0 = blockIdx.x * TBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WN) * 64, wn = (wave % WN) * 64;
  uint4 ra[NA], rb[NB];
  // acc += A B over k in [kb, ke) (phase q: A + ph.aoff[q], B rows mapped)
  auto mainloop = [&](const int q, const int kb, const int ke, v4f (&acc)[4][4]) {
    const bf16_t* __restrict__ Aq = PH ? A + ph.aoff[q] : A;
    auto load = [&](int k0) {
#pragma unroll
      for (int it = 0; it < NA; ++it) {
        const int e = tid + it * NT, r = e >> 3, c = (e & 7) << 3;
        ra[it] = m0 + r < M ? load8(Aq + (int64_t)(m0 + r) * lda, k0 + c, ke, vecA) : make_uint4(0u, 0u, 0u, 0u);
      }
      if constexpr (BKC) {
#pragma unroll
        for (int it = 0; it < NB; ++it) {
          const int e = tid + it * NT, r = e >> 3, c = (e & 7) << 3;
          rb[it] = n0 + r < N ? load8(B + (int64_t)(n0 + r) * ldb, k0 + c, ke, vecB) : make_uint4(0u, 0u, 0u, 0u);
        }
      } else {  // blocks of 4 k x 8 n: k = 4 (e % 16) + r, n = 8 (e / 16) + 0..7
#pragma unroll
        for (int it = 0; it < NB / 4; ++it) {
          const int e = tid + it * NT, kq = (e & 15) << 2, n8 = (e >> 4) << 3;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int gk = k0 + kq + r;
            const int gr = PH ? ph.base[q] + gk + (gk >= ph.run[q] ? ph.gap[q] : 0) : gk;
            rb[4 * it + r] = gk < ke ? load8(B + (int64_t)gr * ldb, n0 + n8, N, vecB) : make_uint4(0u, 0u, 0u, 0u);
          }
        }
      }
    };
    auto stash = [&]() {
#pragma unroll
      for (int it = 0; it < NA; ++it) {
        const int e = tid + it * NT, r = e >> 3, c = (e & 7) << 3;
        *(uint4*)&As[r * GLD + c] = ra[it];
      }
      if constexpr (BKC) {
#pragma unroll
        for (int it = 0; it < NB; ++it) {
          const int e = tid + it * NT, r = e >> 3, c = (e & 7) << 3;
          *(uint4*)&Bs[r * GLD + c] = rb[it];
        }
      } else {
#pragma unroll
        for (int it = 0; it < NB / 4; ++it) {
          const int e = tid + it * NT, kq = (e & 15) << 2, n8 = (e >> 4) << 3;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int d = i >> 1, h = i & 1;
            uint2 v;
            v.x = pick(word(rb[4 * it + 0], d), word(rb[4 * it + 1], d), h);
            v.y = pick(word(rb[4 * it + 2], d), word(rb[4 * it + 3], d), h);
            *(uint2*)&Bs[(n8 + i) * GLD + kq] = v;
          }
        }
      }
    };
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    if (kb < ke) load(kb);
    for (int k0 = kb; k0 < ke; k0 += GBK) {
      __syncthreads();  // the previous stage's fragments are read
      stash();
      __syncthreads();
      if (k0 + GBK < ke) load(k0 + GBK);
#pragma unroll
      for (int kk = 0; kk < GBK; kk += 32) {
        const int kq = kk + 8 * (lane >> 4);
        v8bf a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          a[i] = __builtin_bit_cast(v8bf, *(const uint4*)&As[(wm + i * 16 + (lane & 15)) * GLD + kq]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          b[j] = __builtin_bit_cast(v8bf, *(const uint4*)&Bs[(wn + j * 16 + (lane & 15)) * GLD + kq]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  };
  // result layout of a 16 x 16 tile: lane holds column lane % 16, rows 4 (lane / 16) + r
  if constexpr (!PAIR) {
    const int q = PH ? (int)blockIdx.z : 0;
    const int kb = PH ? 0 : (int)blockIdx.z * kchunk, ke = PH ? ph.K[q] : min(K, kb + kchunk);
    v4f acc[4][4];
    mainloop(q, kb, ke, acc);
    float* Cz = C + (PH ? 0 : (int64_t)blockIdx.z * cz);
    int64_t cof[4];  // column offsets in a row of C
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + wn + j * 16 + (lane & 15);
      cof[j] = gn;
      if (PH) {
        const int hw = ph.Hn * ph.Wn;
        const int b = gn / hw, r = gn - b * hw, y = r / ph.Wn, x = r - y * ph.Wn;
        cof[j] = ((int64_t)b * 2 * ph.Hn + 2 * y + (q >> 1)) * (2 * ph.Wn) + 2 * x + (q & 1);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        if (gm >= M) continue;
        const float bv = (bias && (PH || blockIdx.z == 0)) ? bias[gm] : 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int gn = n0 + wn + j * 16 + (lane & 15);
          if (gn < N) {
            float* c = Cz + (int64_t)gm * ldc + cof[j];
            const float v = (accumulate ? *c : 0.0f) + (acc[i][j][r] + bv);
            *c = relu ? fmaxf(v, 0.0f) : v;
          }
        }
      }
  } else {
    // block z = py: both column phases px = 0, 1 of the row phase, so each
    // output (b, 2y + py, 2x .. 2x + 1) is one 8-byte store
    const int py = (int)blockIdx.z;
    v4f acc0[4][4], acc1[4][4];
    mainloop(2 * py, 0, ph.K[2 * py], acc0);
    __syncthreads();  // LDS reused by the second phase
    mainloop(2 * py + 1, 0, ph.K[2 * py + 1], acc1);
    int64_t cof[4];  // offset of (b, 2y + py, 2x) in a row of C
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + wn + j * 16 + (lane & 15);
      const int hw = ph.Hn * ph.Wn;
      const int b = gn / hw, r = gn - b * hw, y = r / ph.Wn, x = r - y * ph.Wn;
      cof[j] = ((int64_t)b * 2 * ph.Hn + 2 * y + py) * (2 * ph.Wn) + 2 * x;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        if (gm >= M) continue;
        const float bv = bias ? bias[gm] : 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int gn = n0 + wn + j * 16 + (lane & 15);
          if (gn < N) {
            float2* c = (float2*)(C + (int64_t)gm * ldc + cof[j]);
            float2 v = accumulate ? *c : make_float2(0.0f, 0.0f);
            v.x += acc0[i][j][r] + bv;
            v.y += acc1[i][j][r] + bv;
            if (relu) v = make_float2(fmaxf(v.x, 0.0f), fmaxf(v.y, 0.0f));
            *c = v;
          }
        }
      }
  }
}

// col[kidx][p] for kidx = (c, ky, kx) (TM: kidx = (ky, kx, c), tap-major), p
// = (b, oy, ox): the input value under tap (ky, kx) of output (oy, ox), zero
// outside; with up, the input is the
// 2x nearest-neighbour upsampling of x.  x is [b][c][y][x] (nchw) or
// [c][b][y][x].  Grid: y = input channel c, x over pairs of p; each thread
// writes the k^2 rows of its channel for two outputs, each as one 4-byte word
// when P is even (2-byte stores would bind the kernel on store instructions),
// so the input of a channel is read once per pass, not once per tap.  P =
// batch Ho Wo < 2^31 (create checks it): 32-bit index arithmetic.
template <bool NCHW, bool TM>
__global__ __launch_bounds__(EW) void k_im2col(const float* __restrict__ x, int C, int Bt, int H,
                                               int W, int up, int k, int s, int pad, int Ho,
                                               int Wo, bf16_t* __restrict__ col) {
  const int P = Bt * Ho * Wo;
  const int p0 = 2 * (int)(blockIdx.x * EW + threadIdx.x);
  if (p0 >= P) return;
  const int c = blockIdx.y;
  const int He = up ? 2 * H : H, We = up ? 2 * W : W;
  const bool two = p0 + 1 < P;
  int oy[2], ox[2], b[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int p = two ? p0 + e : p0;
    const int q = p / Wo;
    ox[e] = p - q * Wo;
    b[e] = q / Ho;
    oy[e] = q - b[e] * Ho;
  }
  auto value = [&](int e, int ky, int kx) -> float {
    const int iy = oy[e] * s + ky - pad, ix = ox[e] * s + kx - pad;
    if (iy < 0 || iy >= He || ix < 0 || ix >= We) return 0.0f;
    const int sy = up ? iy >> 1 : iy, sx = up ? ix >> 1 : ix;
    const int64_t i = NCHW ? (((int64_t)b[e] * C + c) * H + sy) * W + sx
                           : (((int64_t)c * Bt + b[e]) * H + sy) * W + sx;
    return x[i];
  };
  for (int ky = 0; ky < k; ++ky)
    for (int kx = 0; kx < k; ++kx) {
      const int row = TM ? (ky * k + kx) * C + c : (c * k + ky) * k + kx;
      bf16_t* dst = col + (int64_t)row * P + p0;
      if ((P & 1) == 0) {
        *(uint32_t*)dst = (uint32_t)to_bf16(value(0, ky, kx)) | ((uint32_t)to_bf16(value(1, ky, kx)) << 16);
      } else {
        dst[0] = to_bf16(value(0, ky, kx));
        if (two) dst[1] = to_bf16(value(1, ky, kx));
      }
    }
}

__device__ inline float block_sum(float v, float* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  float t = 0.0f;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

// a = relu(z) (or z) + skip; and a in bfloat16 into a16 (may be null): the
// im2col of a following 1 x 1 layer, whose rows are a's channels.
__global__ __launch_bounds__(EW) void k_act(const float* __restrict__ z, const float* __restrict__ skip,
                                            float* __restrict__ a, int64_t n, int relu,
                                            bf16_t* __restrict__ a16) {
  const int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x;
  if (i >= n) return;
  float v = z[i];
  if (relu) v = fmaxf(v, 0.0f);
  v = skip ? v + skip[i] : v;
  a[i] = v;
  if (a16) a16[i] = to_bf16(v);
}

// dz = da where mask > 0 (relu; the mask is z, or a = relu(z)) or da;
// written to dz and (the GEMM operand) as bfloat16 into dz16 (either may be
// null); the bias gradient's partial sums: block (x, o)
// covers ACT_CHUNK entries of channel o's row (dz is [cout][P]) and writes
// their sum, in a fixed order, to bpart[o][x]; and with a skip input (a =
// act(z) + skip), its gradient: skip_da (+)= da.
constexpr int ACT_PER = 4;                 // entries per thread
constexpr int ACT_CHUNK = EW * ACT_PER;   // entries per block
__global__ __launch_bounds__(EW) void k_act_bwd(const float* __restrict__ da, const float* __restrict__ mask,
                                                float* __restrict__ dz, bf16_t* __restrict__ dz16, int64_t P,
                                                int relu, float* __restrict__ bpart, float* __restrict__ skip_da,
                                                int skip_acc) {
  __shared__ float sh[EW / 64];
  const int o = blockIdx.y;
  const int64_t row = (int64_t)o * P;
  const int64_t p0 = (int64_t)blockIdx.x * ACT_CHUNK + threadIdx.x;
  float sum = 0.0f;
#pragma unroll
  for (int r = 0; r < ACT_PER; ++r) {
    const int64_t p = p0 + (int64_t)r * EW;
    if (p < P) {
      const int64_t i = row + p;
      const float d = da[i];
      if (skip_da) skip_da[i] = skip_acc ? skip_da[i] + d : d;
      const float v = (!relu || mask[i] > 0.0f) ? d : 0.0f;
      if (dz) dz[i] = v;
      if (dz16) dz16[i] = to_bf16(v);
      sum += v;
    }
  }
  sum = block_sum(sum, sh);
  if (threadIdx.x == 0) bpart[(int64_t)o * gridDim.x + blockIdx.x] = sum;
}



// db[o] = sum_p dz[o][p] of every layer from k_act_bwd's partial sums:
// block b is channel b - first[l] of layer l, adding the layer's nchunk
// partial sums of that channel in a fixed order into grad[boff[l] + o].
constexpr int MAXLB = 8;
struct BiasT {
  int64_t bpoff[MAXLB], boff[MAXLB];
  int nchunk[MAXLB], first[MAXLB + 1];
  int nl;
};
__global__ __launch_bounds__(EW) void k_bias_grad(const float* __restrict__ bpart, BiasT t,
                                                  float* __restrict__ grad) {
  __shared__ float sh[EW / 64];
  int l = 0;
  while ((int)blockIdx.x >= t.first[l + 1]) ++l;
  const int o = (int)blockIdx.x - t.first[l];
  const float* row = bpart + t.bpoff[l] + (int64_t)o * t.nchunk[l];
  float v = 0.0f;
  for (int q = threadIdx.x; q < t.nchunk[l]; q += EW) v += row[q];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) grad[t.boff[l] + o] = v;
}

// out[j(i)] = sum_s part[s][i] in a fixed order: wave w of a block adds
// splits w, w + SW, ... of 64 outputs, then the SW wave sums are added in
// wave order.  j(i) = i, or with taps > 0 the canonical weight index of the
// tap-major weight-gradient rows: i = (t cout + o) cin + c -> (o cin + c)
// taps + t.
constexpr int SW = 8;
__global__ __launch_bounds__(64 * SW) void k_sum_splits(const float* __restrict__ part, int S, int64_t n,
                                                        float* __restrict__ out, int taps, int cout,
                                                        int cin) {
  __shared__ float sh[SW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  float v = 0.0f;
  if (i < n)
    for (int s = w; s < S; s += SW) v += part[(int64_t)s * n + i];
  sh[w][lane] = v;
  __syncthreads();
  if (w != 0 || i >= n) return;
  float t = 0.0f;
#pragma unroll
  for (int k = 0; k < SW; ++k) t += sh[k][lane];
  int64_t j = i;
  if (taps > 0) {
    const int64_t oc = (int64_t)cout * cin;
    const int64_t tap = i / oc, r = i - tap * oc;
    j = r * taps + tap;  // r = o cin + c
  }
  out[j] = t;
}

// Backward of a 3 x 3, padding 1 convolution of a 2x nearest-neighbour
// upsampled source (Hs x Ws -> Ho x Wo = 2Hs x 2Ws): the output (Y, X) reads
// source row (Y + ky - 1) / 2, so source row sy receives, through tap ky, the
// output rows 2sy + 1 - ky and 2sy + 2 - ky (those inside [0, Ho)), and
// likewise for columns.  Hence, with the box sums
//   D[t][o][b][sy][sx] = sum of dz[o][b][Y][X] over those 2 x 2 outputs,
//   t = 3 ky + kx,
// the input gradient is dsrc[c][s] = sum_{t, o} W[o][c][t] D[t][o][s] and the
// weight gradient dW[o][c][t] = sum_s D[t][o][s] src[c][s] (s = (b, sy, sx)):
// two GEMMs over the source grid, with no im2col or col2im pass and 1/4 of
// the products of the upsampled grid.  One thread per (o, b, sy, sx) sums
// the 4 x 4 outputs around it into all nine taps; D is bfloat16,
// [9 cout][P4], P4 = batch Hs Ws.
__global__ __launch_bounds__(EW) void k_dmap(const float* __restrict__ dz, int cout, int Bt, int Hs,
                                             int Ws, bf16_t* __restrict__ D) {
  const int pix = (int)(blockIdx.x * EW + threadIdx.x);
  if (pix >= Hs * Ws) return;
  const int o = blockIdx.y, b = blockIdx.z;
  const int sy = pix / Ws, sx = pix - sy * Ws;
  const int Ho = 2 * Hs, Wo = 2 * Ws;
  const float* base = dz + ((int64_t)o * Bt + b) * Ho * Wo;
  float v[4][4];  // rows 2sy - 1 .. 2sy + 2, columns 2sx - 1 .. 2sx + 2
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int Y = 2 * sy - 1 + i, X = 2 * sx - 1 + j;
      v[i][j] = (Y >= 0 && Y < Ho && X >= 0 && X < Wo) ? base[Y * Wo + X] : 0.0f;
    }
  const int64_t P4 = (int64_t)Bt * Hs * Ws;
  const int64_t s = (int64_t)b * Hs * Ws + pix;
#pragma unroll
  for (int ky = 0; ky < 3; ++ky)
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
      // tap ky takes rows i = 2 - ky, 3 - ky of the 4 x 4 block
      const float d = (v[2 - ky][2 - kx] + v[2 - ky][3 - kx]) + (v[3 - ky][2 - kx] + v[3 - ky][3 - kx]);
      D[((int64_t)(3 * ky + kx) * cout + o) * P4 + s] = to_bf16(d);
    }
}

// Input gradient of a 3 x 3, stride-2, padding-1 convolution (input 2Ho x
// 2Wo, output Ho x Wo): input (2y + a, 2x + b) receives output rows y + ey,
// ey in {0, 1}, and columns x + ex, so one stack of dz shifted by (ey, ex),
//   E[(2 ey + ex) cout + o][b][y][x] = dz[o][b][y + ey][x + ex] (0 outside),
// bfloat16, [4 cout][P], P = batch Ho Wo, serves all four phase GEMMs
// (copied from dz in bfloat16).
__global__ __launch_bounds__(EW) void k_emap(const bf16_t* __restrict__ dz, int cout, int Bt, int Ho,
                                             int Wo, bf16_t* __restrict__ E) {
  const int pix = (int)(blockIdx.x * EW + threadIdx.x);
  if (pix >= Ho * Wo) return;
  const int o = blockIdx.y, b = blockIdx.z;
  const int y = pix / Wo, x = pix - y * Wo;
  const bf16_t* base = dz + ((int64_t)o * Bt + b) * Ho * Wo;
  const int64_t P = (int64_t)Bt * Ho * Wo, s = (int64_t)b * Ho * Wo + pix;
#pragma unroll
  for (int ey = 0; ey < 2; ++ey)
#pragma unroll
    for (int ex = 0; ex < 2; ++ex)
      E[((int64_t)(2 * ey + ex) * cout + o) * P + s] =
          (y + ey < Ho && x + ex < Wo) ? base[(y + ey) * Wo + x + ex] : (bf16_t)0;
}

// y is [3][b][hw] (channel-major), t is [b][3][hw]: dy = 2 (y - t) / n and
// per-block partial sums of (y - t)^2 in FP64.
__global__ __launch_bounds__(EW) void k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                             int Bt, int64_t HW, float* __restrict__ dy,
                                             double* __restrict__ part) {
  __shared__ double sh[EW / 64];
  const int64_t n = 3 * (int64_t)Bt * HW;
  const int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x;
  double e2 = 0.0;
  if (i < n) {
    const int64_t hw = i % HW, q = i / HW;
    const int64_t b = q % Bt, c = q / Bt;
    const float d = y[i] - t[(b * 3 + c) * HW + hw];
    dy[i] = 2.0f * d / (float)n;
    e2 = (double)d * d;
  }
  for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = e2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < EW / 64; ++k) s += sh[k];
    part[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(EW) void k_loss_final(const double* __restrict__ part, int64_t nb,
                                                   int64_t n, double* __restrict__ out) {
  __shared__ double sh[EW / 64];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < nb; i += EW) v += part[i];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < EW / 64; ++k) s += sh[k];
    *out = s / (double)n;
  }
}

// [3][b][hw] -> [b][3][hw]
__global__ __launch_bounds__(EW) void k_to_nchw(const float* __restrict__ y, int Bt, int64_t HW,
                                                float* __restrict__ out) {
  const int64_t n = 3 * (int64_t)Bt * HW;
  const int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x;
  if (i >= n) return;
  const int64_t hw = i % HW, q = i / HW;
  const int64_t c = q % 3, b = q / 3;
  out[i] = y[(c * Bt + b) * HW + hw];
}

// Adam with bias correction c1 = 1 - beta1^t, c2 = 1 - beta2^t (the
// bfloat16 GEMM copies of the weights are refreshed by k_prep after it).
__global__ __launch_bounds__(EW) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v, int64_t n,
                                             float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

struct Layer {
  int cin, cout, k, s, up, relu, skip;
  int Hs, Ws;    // source size (before upsampling)
  int Ho, Wo;    // output size
  int64_t woff, boff;
  // bfloat16 GEMM copies of the weights, rows padded to multiples of 8
  // elements (16 bytes): wf[cout][Kp] (forward) and wt[K][coutp] (input
  // gradient), at these element offsets of lbm_no::wf / lbm_no::wt
  int Kp, coutp;
  int64_t wf, wt;
  // upsampling layers: wu[c][Kup] with wu[c][t cout + o] = W[o][c][t] (the
  // input gradient's A operand over the tap-major box sums of k_dmap)
  int Kup;
  int64_t wu;
  // phase GEMM weights (k_gemm PH), four phases of rows of Kph elements at
  // wph: upsampling layers' forward (cout rows, k = (u, v, c)) and stride-2
  // layers' input gradient (cin rows, k = (ey, ex, o)); see k_prep
  int Kph;
  int64_t wph;
  int64_t bpoff;  // the layer's bias-gradient partial sums in lbm_no::bpart
};

// Weight copies of the layers for the GEMMs (see Layer::wf, Layer::wt).
constexpr int MAXL = 8;
struct PrepT {
  int64_t woff[MAXL], wf[MAXL], wt[MAXL], wu[MAXL], wph[MAXL];
  int cout[MAXL], cin[MAXL], K[MAXL], Kp[MAXL], coutp[MAXL], Kup[MAXL], taps[MAXL], Kph[MAXL];
  int kind[MAXL];  // 0 plain, 1 upsampling, 2 stride 2
  int64_t first[MAXL + 1];  // k_prep's flat index: layer l covers [first[l], first[l + 1])
  int nl;
};

// Phase weights of entry j of the four phases q = (a, b) (rows of Kph; the
// row padding stays zero from create).
// Upsampling layer: output (2y + a, 2x + b) reads source rows y + dy with dy
// = floor((a + ky - 1) / 2), i.e. y + a - 1 + u for u in {0, 1}, and likewise
// for columns, so its weights are the sums Weff[o][(u, v, c)] of the W[o][c]
// [ky][kx] that land on (u, v).
// Stride-2 layer, input gradient at (2y + a, 2x + b): the taps with ky = 1
// (a = 0), or ky = 2 and ky = 0 (a = 1), reach output rows y and y + 1 (ey
// = 0, 1), likewise for columns: Wd[c][(ey nx + ex) cout + o] = W[o][c][ky]
// [kx], nx = 1 + b.
__device__ inline void prep_phase(const float* __restrict__ W, const PrepT& t, int l, int64_t j,
                                  bf16_t* __restrict__ wph) {
  const int cin = t.cin[l], cout = t.cout[l], Kph = t.Kph[l];
  const int64_t per = 4 * (int64_t)cin * cout;
  const int q = (int)(j / per), a = q >> 1, b = q & 1;
  const int r = (int)(j - q * per);
  if (t.kind[l] == 1) {
    const int o = r / (4 * cin), kk = r - o * 4 * cin;
    const int u = kk / (2 * cin), v = (kk / cin) & 1, c = kk % cin;
    float sum = 0.0f;
    for (int ky = 0; ky < 3; ++ky)
      for (int kx = 0; kx < 3; ++kx)
        if (((a + ky + 1) >> 1) - 1 == a - 1 + u && ((b + kx + 1) >> 1) - 1 == b - 1 + v)
          sum += W[((int64_t)o * cin + c) * 9 + ky * 3 + kx];
    wph[t.wph[l] + ((int64_t)q * cout + o) * Kph + kk] = to_bf16(sum);
  } else {
    const int c = r / (4 * cout), kk = r - c * 4 * cout;
    const int nx = 1 + b;
    if (kk >= (1 + a) * nx * cout) return;
    const int e = kk / cout, o = kk - e * cout, ey = e / nx, ex = e - ey * nx;
    const int ky = a == 0 ? 1 : (ey == 0 ? 2 : 0), kx = b == 0 ? 1 : (ex == 0 ? 2 : 0);
    wph[t.wph[l] + ((int64_t)q * cin + c) * Kph + kk] = to_bf16(W[((int64_t)o * cin + c) * 9 + ky * 3 + kx]);
  }
}

// One flat index over the layers: in layer l, weight i, rounded to
// bfloat16, into its copies (their padding stays zero from create), then the
// layer's phase weights (prep_phase) for i beyond the weight count.
__global__ __launch_bounds__(EW) void k_prep(const float* __restrict__ par, PrepT t,
                                             bf16_t* __restrict__ wf, bf16_t* __restrict__ wt,
                                             bf16_t* __restrict__ wu, bf16_t* __restrict__ wph) {
  const int64_t g = (int64_t)blockIdx.x * EW + threadIdx.x;
  if (g >= t.first[t.nl]) return;
  int l = 0;
  while (g >= t.first[l + 1]) ++l;
  const int K = t.K[l];
  const int64_t i = g - t.first[l];
  const int64_t nw = (int64_t)t.cout[l] * K;
  if (i >= nw) {
    if (t.kind[l] != 0 && i < nw + 16 * (int64_t)t.cin[l] * t.cout[l]) prep_phase(par + t.woff[l], t, l, i - nw, wph);
    return;
  }
  const int o = (int)(i / K), k = (int)(i - (int64_t)o * K);
  const bf16_t v = to_bf16(par[t.woff[l] + i]);
  wf[t.wf[l] + (int64_t)o * t.Kp[l] + k] = v;
  wt[t.wt[l] + (int64_t)k * t.coutp[l] + o] = v;
  if (t.wu[l] >= 0) {  // k = c taps + tap
    const int c = k / t.taps[l], tap = k - c * t.taps[l];
    wu[t.wu[l] + (int64_t)c * t.Kup[l] + tap * t.cout[l] + o] = v;
  }
}

unsigned grid1(int64_t n) { return (unsigned)((n + EW - 1) / EW); }

// Layers whose convolution runs as phase GEMMs: 1 the forward of a 3 x 3
// convolution of an upsampled source, 2 the input gradient of a 3 x 3
// stride-2 convolution.
int phase_kind(const Layer& l) { return l.k == 3 ? (l.up ? 1 : (l.s == 2 ? 2 : 0)) : 0; }

}  // namespace

struct lbm_no {
  int widths[4];
  int H = 0, W = 0, maxB = 0;
  int64_t npar = 0;
  std::vector<Layer> L;
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  float *par = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  bf16_t *wf = nullptr, *wt = nullptr, *wu = nullptr, *wph = nullptr;  // bfloat16 GEMM copies of the weights (Layer)
  int64_t wf_n = 0, wt_n = 0, wu_n = 0, wph_n = 0, wmax = 0;  // their sizes; k_prep's largest index space
  std::vector<float*> z, a, da;  // per layer, [cout][B][Ho][Wo]
  std::vector<bf16_t*> colL;  // per layer: the forward's im2col, kept for the weight gradient
  bf16_t* col = nullptr;       // work: the backward's box sums (k_dmap) and shifted stacks (k_emap)
  bf16_t* dz16 = nullptr;  // bfloat16 copy of the current layer's dz
  float* split = nullptr;
  int64_t split_n = 0;
  double* lpart = nullptr;
  double* dloss = nullptr;
  float* bpart = nullptr;  // bias-gradient partial sums, [cout][chunks of P]
  long long adam_t = 0;
};

namespace {

// Weight-gradient GEMMs reduce over p = (batch, y, x), hundreds of thousands
// long, into outputs of at most a few hundred x a few thousand: the
// reduction is split so that every layer launches about SPLIT_BLOCKS blocks
// (256 compute units), each split a multiple of GBK long; the partial sums
// are added in split order.
constexpr int SPLIT_BLOCKS = 512;
// GEMM block shape: 64 x 256 outputs for M <= 64 (wm = 1), else 128 x 128.
int gemm_wm(int64_t M) { return M <= 64 ? 1 : 2; }
void wgrad_split(int64_t M, int64_t N, int64_t P, int& S, int64_t& kchunk) {
  const int64_t bm = 64 * gemm_wm(M), bn = 256 / gemm_wm(M);
  const int64_t tiles = ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
  int64_t s = std::max<int64_t>(1, (SPLIT_BLOCKS + tiles - 1) / tiles);
  s = std::min<int64_t>(s, (P + GBK - 1) / GBK);
  kchunk = ((P + s - 1) / s + GBK - 1) / GBK * GBK;
  S = (int)((P + kchunk - 1) / kchunk);
}

void* nalloc(lbm_no* h, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) return nullptr;
  h->allocs.push_back(p);
  return p;
}

void specs(const int* w, int H, int W, std::vector<Layer>& L, int64_t& npar) {
  const int c1 = w[0], c2 = w[1], c3 = w[2], c4 = w[3];
  const int def[8][7] = {{6, c1, 3, 1, 0, 1, -1},  {c1, c2, 3, 2, 0, 1, -1}, {c2, c3, 3, 2, 0, 1, -1},
                         {c3, c4, 3, 2, 0, 1, -1}, {c4, c3, 3, 1, 1, 1, 2},  {c3, c2, 3, 1, 1, 1, 1},
                         {c2, c1, 3, 1, 1, 1, 0},  {c1, 3, 1, 1, 0, 0, -1}};
  L.clear();
  npar = 0;
  int h = H, ww = W;
  for (auto& d : def) {
    Layer l{d[0], d[1], d[2], d[3], d[4], d[5], d[6], h, ww, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, 0, -1, 0};
    const int he = l.up ? 2 * h : h, we = l.up ? 2 * ww : ww;
    const int pad = (l.k - 1) / 2;
    l.Ho = (he + 2 * pad - l.k) / l.s + 1;
    l.Wo = (we + 2 * pad - l.k) / l.s + 1;
    l.woff = npar;
    npar += (int64_t)l.cout * l.cin * l.k * l.k;
    l.boff = npar;
    npar += l.cout;
    L.push_back(l);
    h = l.Ho;
    ww = l.Wo;
  }
}

// C = A B (see k_gemm); A k-contiguous with leading dimension lda >= K.
template <bool BKC>
int gemm(lbm_no* h, int M, int N, int K, const bf16_t* A, int64_t lda, const bf16_t* B, int64_t ldb,
         float* C, int64_t ldc, int64_t cz, int splits, int kchunk, const float* bias, int accumulate = 0,
         int relu = 0) {
  if (M <= 0 || N <= 0 || K <= 0) return LBM_NO_OK;
  if (lda < K || (BKC ? ldb < K : ldb < N) || kchunk < 1 || (splits > 1 && (kchunk % GBK || relu)))
    return fail(LBM_NO_EINVAL, "GEMM operand shapes");
  auto aligned = [](const void* p, int64_t ld) { return ((uintptr_t)p & 15) == 0 && ld % 8 == 0; };
  const int vecA = aligned(A, lda) && kchunk % 8 == 0, vecB = aligned(B, ldb) && (!BKC || kchunk % 8 == 0);
  const int wm = gemm_wm(M), bm = 64 * wm, bn = 256 / wm;
  const dim3 grid((unsigned)((N + bn - 1) / bn), (unsigned)((M + bm - 1) / bm), (unsigned)splits);
  const PhaseT ph{};
  if (wm == 1)
    k_gemm<BKC, 1, false, false><<<grid, NT, 0, h->stream>>>(M, N, K, A, lda, vecA, B, ldb, vecB, C, ldc, cz,
                                                             kchunk, bias, accumulate, ph, relu);
  else
    k_gemm<BKC, 2, false, false><<<grid, NT, 0, h->stream>>>(M, N, K, A, lda, vecA, B, ldb, vecB, C, ldc, cz,
                                                             kchunk, bias, accumulate, ph, relu);
  NOCHK(hipGetLastError());
  return LBM_NO_OK;
}

// The four phase GEMMs of k_gemm PH: M rows, N = batch Hn Wn columns, A =
// four blocks of M rows of lda at A + q M lda, B n-contiguous with ldb, C
// rows of ldc over the 2Hn x 2Wn grid.
int gemm_phases(lbm_no* h, int M, int N, const bf16_t* A, int64_t lda, const bf16_t* B, int64_t ldb,
                float* C, int64_t ldc, const PhaseT& ph, const float* bias, int accumulate, int relu = 0) {
  if (M <= 0 || N <= 0) return LBM_NO_OK;
  for (int q = 0; q < 4; ++q)
    if (ph.K[q] < 1 || ph.K[q] > lda || ph.aoff[q] != (int64_t)q * M * lda)
      return fail(LBM_NO_EINVAL, "phase GEMM operand shapes");
  auto aligned = [](const void* p, int64_t ld) { return ((uintptr_t)p & 15) == 0 && ld % 8 == 0; };
  const int vecA = aligned(A, lda), vecB = aligned(B, ldb);
  const int wm = gemm_wm(M), bm = 64 * wm, bn = 256 / wm;
  const unsigned tiles = (unsigned)(((N + bn - 1) / bn) * ((M + bm - 1) / bm));
  // both column phases per block (contiguous output pairs) when that still
  // gives at least two blocks per compute unit
  const bool pair = 2 * tiles >= 512 && ((uintptr_t)C & 7) == 0 && (ldc & 1) == 0;
  const dim3 grid((unsigned)((N + bn - 1) / bn), (unsigned)((M + bm - 1) / bm), pair ? 2u : 4u);
#define LBM_NO_PH(WMV, PAIRV)                                                                                  \
  k_gemm<false, WMV, true, PAIRV><<<grid, NT, 0, h->stream>>>(M, N, 0, A, lda, vecA, B, ldb, vecB, C, ldc, 0, 0, \
                                                              bias, accumulate, ph, relu)
  if (wm == 1) {
    if (pair) LBM_NO_PH(1, true); else LBM_NO_PH(1, false);
  } else {
    if (pair) LBM_NO_PH(2, true); else LBM_NO_PH(2, false);
  }
#undef LBM_NO_PH
  NOCHK(hipGetLastError());
  return LBM_NO_OK;
}

// Both bfloat16 GEMM copies of every layer's weights from the FP32 master.
int prep_weights(lbm_no* h) {
  PrepT t{};
  const int nl = (int)h->L.size();
  t.first[0] = 0;
  for (int l = 0; l < nl; ++l) {
    const Layer& y = h->L[l];
    t.woff[l] = y.woff;
    t.wf[l] = y.wf;
    t.wt[l] = y.wt;
    t.cout[l] = y.cout;
    t.K[l] = y.cin * y.k * y.k;
    t.Kp[l] = y.Kp;
    t.coutp[l] = y.coutp;
    t.wu[l] = y.wu;
    t.Kup[l] = y.Kup;
    t.taps[l] = y.k * y.k;
    t.cin[l] = y.cin;
    t.wph[l] = y.wph;
    t.Kph[l] = y.Kph;
    t.kind[l] = phase_kind(y);
    t.first[l + 1] = t.first[l] + (int64_t)y.cout * t.K[l] + (t.kind[l] ? 16 * (int64_t)y.cin * y.cout : 0);
  }
  t.nl = nl;
  k_prep<<<grid1(t.first[nl]), EW, 0, h->stream>>>(h->par, t, h->wf, h->wt, h->wu, h->wph);
  NOCHK(hipGetLastError());
  return LBM_NO_OK;
}

int im2col(lbm_no* h, const Layer& l, const float* src, bool nchw, int Bt, bf16_t* col) {
  const int64_t P = (int64_t)Bt * l.Ho * l.Wo;
  const dim3 grid(grid1((P + 1) / 2), (unsigned)l.cin);
  if (nchw)
    k_im2col<true, false><<<grid, EW, 0, h->stream>>>(src, l.cin, Bt, l.Hs, l.Ws, l.up, l.k, l.s, (l.k - 1) / 2, l.Ho, l.Wo, col);
  else
    k_im2col<false, false><<<grid, EW, 0, h->stream>>>(src, l.cin, Bt, l.Hs, l.Ws, l.up, l.k, l.s, (l.k - 1) / 2, l.Ho, l.Wo, col);
  NOCHK(hipGetLastError());
  return LBM_NO_OK;
}

// Forward of an upsampling layer: the tap-major 3 x 3 im2col of the source
// (rows (3 (dy + 1) + dx + 1) cin + c over the source grid), then the four
// phase GEMMs: phase (a, b) reads the taps dy in {a - 1, a}, dx in {b - 1,
// b}, i.e. rows (3a + b) cin + [0, 2 cin) and, 3 cin further on, another
// 2 cin rows.
int forward_up(lbm_no* h, const Layer& l, const float* src, int Bt, bf16_t* col, float* z) {
  const int64_t P4 = (int64_t)Bt * l.Hs * l.Ws;
  const dim3 grid(grid1((P4 + 1) / 2), (unsigned)l.cin);
  k_im2col<false, true><<<grid, EW, 0, h->stream>>>(src, l.cin, Bt, l.Hs, l.Ws, 0, 3, 1, 1, l.Hs, l.Ws, col);
  NOCHK(hipGetLastError());
  PhaseT ph{};
  for (int q = 0; q < 4; ++q) {
    ph.aoff[q] = (int64_t)q * l.cout * l.Kph;
    ph.K[q] = 4 * l.cin;
    ph.base[q] = (3 * (q >> 1) + (q & 1)) * l.cin;
    ph.run[q] = 2 * l.cin;
    ph.gap[q] = l.cin;
  }
  ph.Hn = l.Hs;
  ph.Wn = l.Ws;
  return gemm_phases(h, l.cout, (int)P4, h->wph + l.wph, l.Kph, col, P4, z, (int64_t)Bt * l.Ho * l.Wo, ph,
                     h->par + l.boff, 0);
}

// Input gradient of a stride-2 layer: E = k_emap(dz, bfloat16), then the four phase
// GEMMs into dx (accumulating when it already holds a gradient): phase
// (a, b) takes (1 + a)(1 + b) blocks of cout rows of E, (ey, ex) with ey <=
// a, ex <= b, i.e. rows [0, (1 + b) cout) and, for a = 1, the rows of ey = 1
// from 2 cout on.
int input_grad_s2(lbm_no* h, const Layer& l, const bf16_t* dz, int Bt, float* dx, int accumulate) {
  const int64_t P = (int64_t)Bt * l.Ho * l.Wo;
  k_emap<<<dim3(grid1((int64_t)l.Ho * l.Wo), (unsigned)l.cout, (unsigned)Bt), EW, 0, h->stream>>>(
      dz, l.cout, Bt, l.Ho, l.Wo, h->col);
  NOCHK(hipGetLastError());
  PhaseT ph{};
  for (int q = 0; q < 4; ++q) {
    const int a = q >> 1, b = q & 1;
    ph.aoff[q] = (int64_t)q * l.cin * l.Kph;
    ph.K[q] = (1 + a) * (1 + b) * l.cout;
    ph.base[q] = 0;
    ph.run[q] = (1 + b) * l.cout;
    ph.gap[q] = (1 - b) * l.cout;  // a = 1, b = 0: ey = 1 starts at 2 cout
  }
  ph.Hn = l.Ho;
  ph.Wn = l.Wo;
  return gemm_phases(h, l.cin, (int)P, h->wph + l.wph, l.Kph, h->col, P, dx, (int64_t)Bt * l.Hs * l.Ws, ph,
                     nullptr, accumulate);
}

// A 1 x 1, stride-1 layer: its im2col is its input in bfloat16.
bool pointwise(const Layer& l) { return l.k == 1 && l.s == 1 && !l.up; }

int forward_internal(lbm_no* h, const float* x, int Bt) {
  bool col_ready = false;  // the layer's im2col was written with the previous layer's activation
  for (size_t li = 0; li < h->L.size(); ++li) {
    const Layer& l = h->L[li];
    const int64_t P = (int64_t)Bt * l.Ho * l.Wo;
    const int K = l.cin * l.k * l.k;
    // a layer with a skip input keeps z (the relu mask of its backward) and
    // adds the skip in k_act; any other layer's GEMM writes a = relu(z) (or
    // z) itself, and its backward takes the mask from a (a > 0 exactly where
    // z > 0)
    int rc = LBM_NO_OK;
    if (phase_kind(l) == 1) {
      if (l.skip < 0) return fail(LBM_NO_EINVAL, "upsampling layer without a skip input");
      rc = forward_up(h, l, h->a[li - 1], Bt, h->colL[li], h->z[li]);
    } else {
      if (!col_ready) rc = im2col(h, l, li == 0 ? x : h->a[li - 1], li == 0, Bt, h->colL[li]);
      if (rc) return rc;
      // z[o][p] = W[o][k] col[k][p]: A k-contiguous, B n-contiguous
      float* out = l.skip >= 0 ? h->z[li] : h->a[li];
      rc = gemm<false>(h, l.cout, (int)P, K, h->wf + l.wf, l.Kp, h->colL[li], P, out, P, 0, 1, K,
                       h->par + l.boff, 0, l.skip >= 0 ? 0 : l.relu);
    }
    if (rc) return rc;
    const bool next_pw = li + 1 < h->L.size() && pointwise(h->L[li + 1]);
    col_ready = false;
    if (l.skip >= 0) {
      const int64_t n = (int64_t)l.cout * P;
      k_act<<<grid1(n), EW, 0, h->stream>>>(h->z[li], h->a[l.skip], h->a[li], n, l.relu,
                                            next_pw ? h->colL[li + 1] : nullptr);
      NOCHK(hipGetLastError());
      col_ready = next_pw;
    }
  }
  return LBM_NO_OK;
}

int check_batch(lbm_no* h, int Bt) {
  if (!h) return fail(LBM_NO_EINVAL, "null handle");
  if (Bt < 1 || Bt > h->maxB) return fail(LBM_NO_EINVAL, "batch out of [1, max_batch]");
  return LBM_NO_OK;
}

// Host-side failures (allocation) become error codes: nothing may unwind
// through the C ABI.
template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(LBM_NO_ENOMEM, "host memory exhausted");
  } catch (const std::exception& e) {
    return fail(LBM_NO_EDEVICE, e.what());
  }
}

}  // namespace

extern "C" {

const char* lbm_no_last_error(void) { return g_err.c_str(); }

int lbm_no_param_count(const int32_t* widths, int64_t* count) {
  if (!widths || !count) return fail(LBM_NO_EINVAL, "null argument");
  for (int i = 0; i < 4; ++i)
    if (widths[i] < 1 || widths[i] > 1024) return fail(LBM_NO_EINVAL, "widths out of [1, 1024]");
  std::vector<Layer> L;
  int w[4] = {widths[0], widths[1], widths[2], widths[3]};
  specs(w, 8, 8, L, *count);
  return LBM_NO_OK;
}

void lbm_no_destroy(lbm_no* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  for (void* p : h->allocs) (void)hipFree(p);
  delete h;
}

int lbm_no_create(const int32_t* widths, int32_t height, int32_t width, int32_t max_batch,
                  const float* params, void* hip_stream, lbm_no** out) {
  return guarded([&]() -> int {
    if (out) *out = nullptr;
    if (!widths || !params || !out) return fail(LBM_NO_EINVAL, "null argument");
    for (int i = 0; i < 4; ++i)
      if (widths[i] < 2 || widths[i] > 1024 || (widths[i] & 1))
        return fail(LBM_NO_EINVAL, "widths must be even, in [2, 1024]");
    if (height < 8 || width < 8 || height > 2048 || width > 2048 || height % 8 || width % 8)
      return fail(LBM_NO_EINVAL, "height and width must be multiples of 8 in [8, 2048]");
    if (max_batch < 1 || (int64_t)max_batch * height * width > (1ll << 31) / 64)
      return fail(LBM_NO_EINVAL, "max_batch out of range");
    lbm_no* h = new lbm_no();
    auto bail = [&](int rc) {
      lbm_no_destroy(h);
      return rc;
    };
    for (int i = 0; i < 4; ++i) h->widths[i] = widths[i];
    h->H = height;
    h->W = width;
    h->maxB = max_batch;
    specs(h->widths, height, width, h->L, h->npar);
    h->stream = (hipStream_t)hip_stream;  // NULL: the null stream (torch's default stream)
    const size_t np = (size_t)h->npar;
    h->par = (float*)nalloc(h, np * 4);
    h->grad = (float*)nalloc(h, np * 4);
    h->m = (float*)nalloc(h, np * 4);
    h->v = (float*)nalloc(h, np * 4);
    for (Layer& l : h->L) {
      const int K = l.cin * l.k * l.k;
      l.Kp = (K + 7) / 8 * 8;
      l.coutp = (l.cout + 7) / 8 * 8;
      l.wf = h->wf_n;
      l.wt = h->wt_n;
      h->wf_n += (int64_t)l.cout * l.Kp;
      h->wt_n += (int64_t)K * l.coutp;
      int64_t nprep = (int64_t)l.cout * K;
      if (l.up) {
        l.Kup = (l.k * l.k * l.cout + 7) / 8 * 8;
        l.wu = h->wu_n;
        h->wu_n += (int64_t)l.cin * l.Kup;
      }
      if (phase_kind(l)) {
        l.Kph = (4 * (l.up ? l.cin : l.cout) + 7) / 8 * 8;
        l.wph = h->wph_n;
        h->wph_n += 4 * (int64_t)(l.up ? l.cout : l.cin) * l.Kph;
        nprep += 16 * (int64_t)l.cin * l.cout;
      }
      h->wmax = std::max(h->wmax, nprep);
    }
    h->wf = (bf16_t*)nalloc(h, (size_t)h->wf_n * 2);
    h->wt = (bf16_t*)nalloc(h, (size_t)h->wt_n * 2);
    h->wu = (bf16_t*)nalloc(h, (size_t)h->wu_n * 2);
    h->wph = (bf16_t*)nalloc(h, (size_t)h->wph_n * 2);
    if (!h->par || !h->grad || !h->m || !h->v || !h->wf || !h->wt || !h->wu || !h->wph)
      return bail(fail(LBM_NO_ENOMEM, "parameters"));
    NOCHK(hipMemsetAsync(h->wf, 0, (size_t)h->wf_n * 2, h->stream));  // row padding stays zero
    NOCHK(hipMemsetAsync(h->wt, 0, (size_t)h->wt_n * 2, h->stream));
    NOCHK(hipMemsetAsync(h->wu, 0, (size_t)h->wu_n * 2, h->stream));
    NOCHK(hipMemsetAsync(h->wph, 0, (size_t)h->wph_n * 2, h->stream));
    int64_t colmax = 0, splitmax = 0, actmax = 0, bpmax = 0;
    for (size_t li = 0; li < h->L.size(); ++li) {
      const Layer& l = h->L[li];
      const int64_t P = (int64_t)max_batch * l.Ho * l.Wo;
      const size_t n = (size_t)l.cout * P * 4;
      actmax = std::max(actmax, (int64_t)l.cout * P);
      float* zl = (float*)nalloc(h, n);
      float* al = (float*)nalloc(h, n);
      float* dl = (float*)nalloc(h, n);
      if (!zl || !al || !dl) return bail(fail(LBM_NO_ENOMEM, "activations"));
      h->z.push_back(zl);
      h->a.push_back(al);
      h->da.push_back(dl);
      const int64_t K = (int64_t)l.cin * l.k * l.k;
      // the forward's im2col, kept: over the source grid for upsampling layers
      const int64_t ncol = l.up ? 9 * l.cin * (int64_t)max_batch * l.Hs * l.Ws : K * P;
      bf16_t* cl = (bf16_t*)nalloc(h, (size_t)ncol * 2);
      if (!cl) return bail(fail(LBM_NO_ENOMEM, "im2col buffers"));
      h->colL.push_back(cl);
      if (phase_kind(l) == 2) colmax = std::max(colmax, 4 * l.cout * P);  // k_emap's stack
      int S;
      int64_t kchunk;
      wgrad_split(l.cout, K, P, S, kchunk);
      splitmax = std::max(splitmax, (int64_t)S * l.cout * K);
      if (l.up) {  // box sums in col, split partials of the tap-major weight gradient
        const int64_t P4 = (int64_t)max_batch * l.Hs * l.Ws;
        colmax = std::max(colmax, 9 * l.cout * P4);
        wgrad_split(9 * l.cout, l.cin, P4, S, kchunk);
        splitmax = std::max(splitmax, (int64_t)S * 9 * l.cout * l.cin);
      }
      h->L[li].bpoff = bpmax;  // the layers' partial sums side by side
      bpmax += (int64_t)l.cout * ((P + ACT_CHUNK - 1) / ACT_CHUNK);
    }
    h->col = (bf16_t*)nalloc(h, (size_t)colmax * 2);
    h->dz16 = (bf16_t*)nalloc(h, (size_t)actmax * 2);
    h->split = (float*)nalloc(h, (size_t)splitmax * 4);
    h->split_n = splitmax;
    const int64_t lb = (3 * (int64_t)max_batch * height * width + EW - 1) / EW;
    h->lpart = (double*)nalloc(h, (size_t)lb * 8);
    h->dloss = (double*)nalloc(h, 8);
    h->bpart = (float*)nalloc(h, (size_t)bpmax * 4);
    if (!h->col || !h->dz16 || !h->split || !h->lpart || !h->dloss || !h->bpart)
      return bail(fail(LBM_NO_ENOMEM, "work space"));
    const int rc = lbm_no_set_params(h, params);
    if (rc) return bail(rc);
    *out = h;
    return LBM_NO_OK;
  });
}

int lbm_no_set_params(lbm_no* h, const float* params) {
  return guarded([&]() -> int {
    if (!h || !params) return fail(LBM_NO_EINVAL, "null argument");
    const size_t np = (size_t)h->npar;
    NOCHK(hipMemcpyAsync(h->par, params, np * 4, hipMemcpyHostToDevice, h->stream));
    NOCHK(hipMemsetAsync(h->m, 0, np * 4, h->stream));
    NOCHK(hipMemsetAsync(h->v, 0, np * 4, h->stream));
    NOCHK(hipMemsetAsync(h->grad, 0, np * 4, h->stream));
    const int rc = prep_weights(h);
    if (rc) return rc;
    NOCHK(hipStreamSynchronize(h->stream));
    h->adam_t = 0;
    return LBM_NO_OK;
  });
}

int lbm_no_forward(lbm_no* h, const float* x, int32_t batch, float* y) {
  return guarded([&]() -> int {
    int rc = check_batch(h, batch);
    if (rc) return rc;
    if (!x || !y) return fail(LBM_NO_EINVAL, "null tensor");
    rc = forward_internal(h, x, batch);
    if (rc) return rc;
    const int64_t HW = (int64_t)h->H * h->W;
    k_to_nchw<<<grid1(3 * batch * HW), EW, 0, h->stream>>>(h->a.back(), batch, HW, y);
    NOCHK(hipGetLastError());
    return LBM_NO_OK;
  });
}

int lbm_no_gradients(lbm_no* h, const float* x, const float* target, int32_t batch, double* loss) {
  return guarded([&]() -> int {
    int rc = check_batch(h, batch);
    if (rc) return rc;
    if (!x || !target) return fail(LBM_NO_EINVAL, "null tensor");
    rc = forward_internal(h, x, batch);
    if (rc) return rc;
    const int nl = (int)h->L.size();
    const int64_t HW = (int64_t)h->H * h->W;
    const int64_t nout = 3 * (int64_t)batch * HW;
    const int64_t nb = (nout + EW - 1) / EW;
    k_loss<<<(unsigned)nb, EW, 0, h->stream>>>(h->a[nl - 1], target, batch, HW, h->da[nl - 1], h->lpart);
    NOCHK(hipGetLastError());
    k_loss_final<<<1, EW, 0, h->stream>>>(h->lpart, nb, nout, h->dloss);
    NOCHK(hipGetLastError());
    std::vector<char> have(nl, 0);  // activation gradient already written
    have[nl - 1] = 1;
    for (int li = nl - 1; li >= 0; --li) {
      const Layer& l = h->L[li];
      const int64_t P = (int64_t)batch * l.Ho * l.Wo;
      const int K = l.cin * l.k * l.k;
      // dz over z (and the bias gradient's partial sums); the skip passes da on unchanged
      const unsigned nchunk = (unsigned)((P + ACT_CHUNK - 1) / ACT_CHUNK);
      float* skip_da = l.skip >= 0 ? h->da[l.skip] : nullptr;
      // the relu mask: z where the layer has a skip input, else a (= relu(z)); dz over z
      const float* mask = l.skip >= 0 ? h->z[li] : h->a[li];
      // FP32 dz for the box sums of an upsampling layer, else bfloat16 dz for the GEMMs
      k_act_bwd<<<dim3(nchunk, (unsigned)l.cout), EW, 0, h->stream>>>(h->da[li], mask, l.up ? h->z[li] : nullptr,
                                                                       l.up ? nullptr : h->dz16, P, l.relu,
                                                                       h->bpart + l.bpoff, skip_da,
                                                                       l.skip >= 0 ? have[l.skip] : 0);
      NOCHK(hipGetLastError());
      if (l.skip >= 0) have[l.skip] = 1;
      int S;
      int64_t kchunk;
      if (l.up) {
        // 3 x 3 convolution of an upsampled source (li > 0): both gradients
        // over the source grid from the box sums D = k_dmap(dz) (in col)
        const int64_t P4 = (int64_t)batch * l.Hs * l.Ws;
        const int M9 = 9 * l.cout;
        k_dmap<<<dim3(grid1((int64_t)l.Hs * l.Ws), (unsigned)l.cout, (unsigned)batch), EW, 0, h->stream>>>(
            h->z[li], l.cout, batch, l.Hs, l.Ws, h->col);
        NOCHK(hipGetLastError());
        // dW[o][c][t] = sum_s D[t cout + o][s] src[c][s]: A = D, B k(=s)-contiguous, the
        // source in bfloat16 being the centre tap (rows 4 cin ..) of the forward's im2col
        wgrad_split(M9, l.cin, P4, S, kchunk);
        const int64_t mn = (int64_t)M9 * l.cin;
        if ((int64_t)S * mn > h->split_n) return fail(LBM_NO_EINVAL, "split work space too small");
        rc = gemm<true>(h, M9, l.cin, (int)P4, h->col, P4, h->colL[li] + 4 * l.cin * P4, P4, h->split, l.cin, mn,
                        S, (int)kchunk, nullptr);
        if (rc) return rc;
        k_sum_splits<<<(unsigned)((mn + 63) / 64), 64 * SW, 0, h->stream>>>(h->split, S, mn, h->grad + l.woff, 9,
                                                                         l.cout, l.cin);
        NOCHK(hipGetLastError());
        // da[li - 1][c][s] (+)= sum_{t, o} W[o][c][t] D[t cout + o][s]: A = wu, B = D n(=s)-contiguous
        rc = gemm<false>(h, l.cin, (int)P4, M9, h->wu + l.wu, l.Kup, h->col, P4, h->da[li - 1], P4, 0, 1, M9,
                         nullptr, have[li - 1]);
        if (rc) return rc;
        have[li - 1] = 1;
        continue;
      }
      // weight gradient over the forward's im2col, split over p, partials summed in order
      wgrad_split(l.cout, K, P, S, kchunk);
      const int64_t mn = (int64_t)l.cout * K;
      if ((int64_t)S * mn > h->split_n) return fail(LBM_NO_EINVAL, "split work space too small");
      // dW[o][k] = dz[o][p] col[k][p]: A k(=p)-contiguous, B k(=p)-contiguous
      rc = gemm<true>(h, l.cout, K, (int)P, h->dz16, P, h->colL[li], P, h->split, K, mn, S, (int)kchunk, nullptr);
      if (rc) return rc;
      k_sum_splits<<<(unsigned)((mn + 63) / 64), 64 * SW, 0, h->stream>>>(h->split, S, mn, h->grad + l.woff, 0, 0,
                                                                       0);
      NOCHK(hipGetLastError());
      if (li == 0) break;  // no gradient with respect to the input
      if (l.k == 1 && l.s == 1) {  // 1 x 1: the input gradient is the GEMM itself
        rc = gemm<false>(h, K, (int)P, l.cout, h->wt + l.wt, l.coutp, h->dz16, P, h->da[li - 1], P, 0, 1, l.cout,
                         nullptr, have[li - 1]);
        if (rc) return rc;
        have[li - 1] = 1;
        continue;
      }
      if (phase_kind(l) == 2) {
        rc = input_grad_s2(h, l, h->dz16, batch, h->da[li - 1], have[li - 1]);
        if (rc) return rc;
        have[li - 1] = 1;
        continue;
      }
      // every layer with an input gradient is upsampling, stride 2 or 1 x 1 (specs)
      return fail(LBM_NO_EINVAL, "no input-gradient path for this layer");
    }
    // every layer's bias gradient from its partial sums, one launch
    BiasT bt{};
    bt.first[0] = 0;
    for (int li = 0; li < nl; ++li) {
      const Layer& l = h->L[li];
      const int64_t P = (int64_t)batch * l.Ho * l.Wo;
      bt.bpoff[li] = l.bpoff;
      bt.boff[li] = l.boff;
      bt.nchunk[li] = (int)((P + ACT_CHUNK - 1) / ACT_CHUNK);
      bt.first[li + 1] = bt.first[li] + l.cout;
    }
    bt.nl = nl;
    k_bias_grad<<<(unsigned)bt.first[nl], EW, 0, h->stream>>>(h->bpart, bt, h->grad);
    NOCHK(hipGetLastError());
    if (loss) {
      NOCHK(hipMemcpyAsync(loss, h->dloss, 8, hipMemcpyDeviceToHost, h->stream));
      NOCHK(hipStreamSynchronize(h->stream));
    }
    return LBM_NO_OK;
  });
}

int lbm_no_adam(lbm_no* h, float lr, float beta1, float beta2, float eps) {
  return guarded([&]() -> int {
    if (!h || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
      return fail(LBM_NO_EINVAL, "bad handle or Adam hyper-parameters");
    h->adam_t += 1;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)h->adam_t));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)h->adam_t));
    k_adam<<<grid1(h->npar), EW, 0, h->stream>>>(h->par, h->grad, h->m, h->v, h->npar, lr, beta1, beta2, eps, c1,
                                                 c2);
    NOCHK(hipGetLastError());
    return prep_weights(h);
  });
}

int lbm_no_get(lbm_no* h, int32_t which, float* host_out) {
  return guarded([&]() -> int {
    if (!h || !host_out || which < 0 || which > 1) return fail(LBM_NO_EINVAL, "bad argument");
    NOCHK(hipMemcpyAsync(host_out, which == 0 ? h->par : h->grad, (size_t)h->npar * 4, hipMemcpyDeviceToHost,
                         h->stream));
    NOCHK(hipStreamSynchronize(h->stream));
    return LBM_NO_OK;
  });
}

int lbm_no_sync(lbm_no* h) {
  if (!h) return fail(LBM_NO_EINVAL, "null handle");
  NOCHK(hipStreamSynchronize(h->stream));
  return LBM_NO_OK;
}

}  // extern "C"
