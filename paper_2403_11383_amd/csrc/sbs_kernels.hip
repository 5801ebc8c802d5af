// sbs_kernels.hip -- gfx950 kernels of one SBS control step.
//
// Stages of one iteration (Alg. 1: sampling, evaluation, sorting, update),
// each one launch over every controller of a fused batch:
//   k_noise    counter-based Gaussian noise z[j][k][12] and gait-frequency
//              increments q[k] (Sampling)
//   k_rollout  one lane per sample: SRBD rollout of Eq. (1) with explicit
//              Euler, world-fixed footholds placed by Eq. (2) at touchdown,
//              quadratic cost of Sec. V (Alg. 2, Evaluation); k_rollout_quad
//              is the same rollout on four lanes per sample (one per leg)
//   k_select   elite and best-sample controllers, one workgroup per
//              controller: lowest cost, top-K_e radix selection (Alg. 1) or
//              the best sample (Alg. 3), frequency moments (Sorting)
//   k_update   elite and best-sample controllers, one workgroup per
//              (controller, step): FP64 moments of the chosen noise rows,
//              new mean and elite std; step 0 of the last iteration writes
//              the action (Update)
//   k_update_mppi  MPPI controllers, one workgroup per (controller, step):
//              log-sum-exp weighting with an FP64 normaliser and the
//              weighted noise sum fused (Alg. 4); step 0 writes the
//              per-iteration scalars and, last, the action
// The warm-started mean (Sec. III-A) is the previous tick's mean read one
// step (or knot) shifted by the next reader.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <functional>
#include <limits>
#include <type_traits>

#include "sbs_device.h"

namespace sbs {

// ---------------------------------------------------------------------------
// Noise contract: Philox4x32-10 keyed by the seed, counter (k, j, tick,
// (r << 8) | call); calls 0..2 give the six Box-Muller pairs of row j (pair
// p from words 2 (p mod 2), +1 of call p / 2), pair p serving one force
// component of the two legs of a diagonal: pairs 0..2 the x, y, z forces of
// legs 0 and 3 (dims 0..2, 9..11), pairs 3..5 those of legs 1 and 2 (dims
// 3..5, 6..8); call 3 at j = 0 the frequency.  Gaussians by Box-Muller on 24-bit uniforms with a
// fixed sequence of IEEE FP32 operations (no contraction), so the result is
// reproducible bit for bit on any IEEE machine.
// ---------------------------------------------------------------------------
// a ^ b ^ k in one VALU instruction: gfx950's three-input bitwise operation
// with truth table 0x96 (odd parity).  The key word k is wave-uniform and is
// read from a scalar register.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

// The key (k0, k1) must be uniform across the wave (one controller's seed).
__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                              uint32_t &c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = xor3_key((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3_key((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// IEEE round-to-nearest square root for the Box-Muller radius, whose
// argument is -0, +0 or in [2^-24, 34]: the hardware root (within one ulp)
// moved to a neighbour where that neighbour's residual says it is closer.
// No scaling is needed because the argument never comes near the tiny
// inputs where the hardware root loses accuracy.  For a zero argument the
// neighbour tests fail (NaN or signed-zero residuals), and the root keeps
// the argument's sign.
__device__ __forceinline__ float sqrt_rn_radius(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float sd = __uint_as_float(__float_as_uint(s) - 1u);
  const float su = __uint_as_float(__float_as_uint(s) + 1u);
  const float rd = __builtin_fmaf(-sd, s, x);
  const float ru = __builtin_fmaf(-su, s, x);
  const float r = (rd <= 0.0f) ? sd : s;
  return (ru > 0.0f) ? su : r;
}

__device__ __forceinline__ float2 gauss_pair(uint32_t w0, uint32_t w1) {
#pragma clang fp contract(off)
  const uint32_t i1 = (w0 >> 8) + 1u;   // u1 = i1 2^-24 in (0, 1]
  const uint32_t i2 = w1 >> 8;          // u2 = i2 2^-24 in [0, 1)
  // i1 = 2^e m, m in [1, 2): the exponent and fraction fields of i1
  // converted to FP32 (exact: i1 <= 2^24)
  const uint32_t fb = __float_as_uint((float)i1);
  int e = (int)(fb >> 23) - 127;
  float m = __uint_as_float((fb & 0x7FFFFFu) | 0x3F800000u);
  const bool above = m > 0x1.6a09e6p+0f;  // fold onto [sqrt(2)/2, sqrt(2)]
  m = above ? m * 0.5f : m;
  e = above ? e + 1 : e;
  // ln m = f + f^2 (f P(f) - 1/2), f = m - 1 (exact), P of degree 7 fitted
  // to (ln(1 + f) - f + f^2 / 2) / f^3 on the folded range: no division
  const float f = m - 1.0f;
  const float h = f * f;
  float p = __builtin_fmaf(f, -0x1.38b4e6p-4f, 0x1.055b58p-3f);
  p = __builtin_fmaf(f, p, -0x1.0d8556p-3f);
  p = __builtin_fmaf(f, p, 0x1.22da20p-3f);
  p = __builtin_fmaf(f, p, -0x1.547242p-3f);
  p = __builtin_fmaf(f, p, 0x1.99a008p-3f);
  p = __builtin_fmaf(f, p, -0x1.000228p-2f);
  p = __builtin_fmaf(f, p, 0x1.555554p-2f);
  const float lnm = __builtin_fmaf(h, __builtin_fmaf(f, p, -0.5f), f);
  const float ke = (float)(e - 24);
  const float lnu = __builtin_fmaf(ke, 0x1.62e4p-1f, __builtin_fmaf(ke, 0x1.7f7d1cp-20f, lnm));
  const float rho = sqrt_rn_radius(-2.0f * lnu);

  const uint32_t n = (i2 + (1u << 21)) >> 22;
  const int32_t fi = (int32_t)i2 - (int32_t)(n << 22);
  const float a = (float)fi * 0x1p-24f;
  const float a2 = a * a;
  float ps = __builtin_fmaf(a2, 0x1.507834p+5f, -0x1.32d2ccp+6f);
  ps = __builtin_fmaf(a2, ps, 0x1.466bc6p+6f);
  ps = __builtin_fmaf(a2, ps, -0x1.4abbcep+5f);
  ps = __builtin_fmaf(a2, ps, 0x1.921fb6p+2f);
  const float sn = a * ps;
  float pc = __builtin_fmaf(a2, -0x1.a6d1f2p+4f, 0x1.e1f506p+5f);
  pc = __builtin_fmaf(a2, pc, -0x1.55d3c8p+6f);
  pc = __builtin_fmaf(a2, pc, 0x1.03c1f0p+6f);
  pc = __builtin_fmaf(a2, pc, -0x1.3bd3ccp+4f);
  const float cs = __builtin_fmaf(a2, pc, 1.0f);
  // quadrant by rotation: quadrant 1 maps (cos, sin) to (-sin, cos), 2 to
  // (-cos, -sin), 3 to (sin, -cos); the negations are sign-bit flips
  const uint32_t quad = n & 3u;
  const bool swap = (quad & 1u) != 0u;
  const float c0 = swap ? sn : cs, s0 = swap ? cs : sn;
  const float c = __uint_as_float(__float_as_uint(c0) ^ (((quad + 1u) & 2u) << 30));
  const float sv = __uint_as_float(__float_as_uint(s0) ^ ((quad & 2u) << 30));
  return make_float2(rho * c, rho * sv);
}

__device__ __forceinline__ uint32_t q_of_freq(double f, double dt) {
#pragma clang fp contract(off)
  const double v = __builtin_rint((f * dt) * 4294967296.0);
  if (!(v > 0.0)) return 0u;
  if (v > 4294967295.0) return 4294967295u;
  return (uint32_t)v;
}

__device__ __forceinline__ uint32_t freq_gaussian(double mf, double sf, float z, double fmin,
                                                  double fmax, double dt) {
#pragma clang fp contract(off)
  const double prod = sf * (double)z;
  double f = mf + prod;
  f = (f < fmin) ? fmin : f;
  f = (f > fmax) ? fmax : f;
  return q_of_freq(f, dt);
}

// Item of flattened block b: the largest i < n with start[i] <= b, start
// being a stage's non-decreasing block prefix sums (n + 1 entries).  Every
// lane of the wave tests one boundary and a ballot counts those <= b: one
// memory round trip for n < 64, two (coarse, then fine) up to 4032 items, a
// binary search inside the coarse segment beyond.  Called by whole waves.
__device__ __forceinline__ int find_item(const int32_t *start, int n, int b) {
  const int lane = threadIdx.x & 63;
  if (n < 64) {
    const bool le = lane <= n && start[lane] <= b;
    return (int)__popcll(__ballot(le)) - 1;
  }
  const int step = (n + 64) / 64;  // 64 coarse boundaries cover all n + 1
  const int i0 = lane * step;
  const int c = (int)__popcll(__ballot(i0 <= n && start[i0] <= b)) - 1;
  const int base = c * step;
  if (step <= 64) {
    const int i1 = base + lane;
    return base + (int)__popcll(__ballot(lane < step && i1 <= n && start[i1] <= b)) - 1;
  }
  int lo = base, hi = base + step < n ? base + step : n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The descriptor of a single-controller launch, read in place from the
// kernel-argument segment, where it follows the LaunchTab argument (explicit
// arguments are laid out in order at their natural alignment).  Naming the
// by-value parameter instead lets the compiler copy the whole descriptor into
// per-lane scratch whenever a field's address meets a global address in a
// conditional choice.
__device__ __forceinline__ const TickDesc &inline_desc() {
  constexpr size_t kOff =
      (sizeof(LaunchTab) + alignof(TickDesc) - 1) / alignof(TickDesc) * alignof(TickDesc);
  const char *seg = (const char *)__builtin_amdgcn_kernarg_segment_ptr();
  return *reinterpret_cast<const TickDesc *>(seg + kOff);
}

// A launch either carries one controller's descriptor by value (INL, the
// latency path of a single controller: no descriptor copy) or indexes the
// batch's descriptor array through the stage's block map.
template <bool INL>
__device__ __forceinline__ int stage_item(const int32_t *start, int n, int b) {
  return INL ? 0 : find_item(start, n, b);
}
template <bool INL>
__device__ __forceinline__ int stage_start(const int32_t *start, int i) {
  return INL ? 0 : start[i];
}

// Gait-frequency draw of sample k in iteration r (Sec. IV-C): the fixed
// increment, a uniform integer increment on [q_lo, q_hi] from Philox word 0
// of call 3, or a Gaussian around the running frequency mean, clamped and
// quantised in FP64 without contraction.
__device__ __forceinline__ uint32_t draw_q(const TickDesc &d, int r, int k) {
  if (d.freq_mode == 0) return d.q_fixed;
  uint32_t c0 = (uint32_t)k, c1 = 0u, c2 = d.tick, c3 = ((uint32_t)r << 8) | 3u;
  philox4x32_10(c0, c1, c2, c3, (uint32_t)d.seed, (uint32_t)(d.seed >> 32));
  if (d.freq_mode == 1) {
    const uint64_t span = (uint64_t)(d.q_hi - d.q_lo) + 1u;
    return d.q_lo + (uint32_t)(((uint64_t)c0 * span) >> 32);
  }
  if (d.freq_mode == 3) {  // one member of the frequency set, each with probability 1/n
    const uint32_t i = (uint32_t)(((uint64_t)c0 * (uint64_t)d.n_fset) >> 32);
    return d.q_set[i];
  }
  const double mf = (r == 0) ? d.ctl[0] : d.it[IT_MUF];
  const double sf = (r == 0) ? d.sigma_f0 : d.it[IT_SIGF];
  return freq_gaussian(mf, sf, gauss_pair(c0, c1).x, d.f_min, d.f_max, d.dt);
}

// Noise row j of sample k in iteration r: the 12 Gaussians of the GRF
// dimensions, from Philox calls 0..2 of the counter (k, j, tick, (r << 8) |
// call): pair p of words 2 (p mod 2), +1 of call p / 2 goes to dims
// kPairDim[p] (the same force component of the two legs of a diagonal).
__device__ __forceinline__ void noise_row(uint32_t key0, uint32_t key1, uint32_t rw,
                                          uint32_t tick, uint32_t k, uint32_t j, float z[12]) {
  constexpr int kPairDim[6][2] = {{0, 9}, {1, 10}, {2, 11}, {3, 6}, {4, 7}, {5, 8}};
#pragma unroll
  for (uint32_t call = 0; call < 3; ++call) {
    uint32_t c0 = k, c1 = j, c2 = tick, c3 = rw | call;
    philox4x32_10(c0, c1, c2, c3, key0, key1);
    const float2 ga = gauss_pair(c0, c1);
    const float2 gb = gauss_pair(c2, c3);
    z[kPairDim[2 * call][0]] = ga.x;
    z[kPairDim[2 * call][1]] = ga.y;
    z[kPairDim[2 * call + 1][0]] = gb.x;
    z[kPairDim[2 * call + 1][1]] = gb.y;
  }
}

// GRF noise of iterations tab.r .. tab.r + tab.r_count - 1: one thread per
// (iteration, row j, sample k), a row being a step or a spline knot;
// iteration r lands at z + r * z_iter_stride.  The noise depends only on
// (seed, tick, r, k, j), never on the state, so it can be produced ahead of
// the tick that consumes it.
template <bool INL>
__global__ void __launch_bounds__(kNoiseBlock) k_noise(LaunchTab tab, TickDesc inl) {
  const int per_iter = tab.total_noise;
  const int rr = blockIdx.x / per_iter;
  const int b = blockIdx.x - rr * per_iter;
  const int i = stage_item<INL>(tab.noise_start, tab.n, b);
  const TickDesc &d = INL ? inline_desc() : tab.desc[tab.item[i]];
  const int local = b - stage_start<INL>(tab.noise_start, i);
  const int nkb = (d.N + kNoiseBlock - 1) / kNoiseBlock;
  const int jb = local / nkb;
  const int k = (local - jb * nkb) * kNoiseBlock + (int)threadIdx.x;
  if (k >= d.N) return;
  const int r = tab.r + rr;
  // descriptor fields in registers: the noise stores could alias the
  // descriptor for all the compiler knows, which would reload them per row
  const uint32_t key0 = (uint32_t)d.seed, key1 = (uint32_t)(d.seed >> 32);
  const uint32_t rw = (uint32_t)r << 8, tick = d.tick;
  const int N = d.N;
  float *zr = d.z + (size_t)r * d.z_iter_stride;
  // rows jb * rpt .. jb * rpt + rpt - 1 of sample k (rpt = 1 in batched
  // launches; a single controller's ahead-of-time noise uses fewer, longer
  // waves so that it leaves more of the chip to the tick in flight)
  const int rpt = tab.noise_rpt > 1 ? tab.noise_rpt : 1;
  const int j0 = jb * rpt, j1 = j0 + rpt < d.M ? j0 + rpt : d.M;
  for (int j = j0; j < j1; ++j) {
    float z[12];
    noise_row(key0, key1, rw, tick, (uint32_t)k, (uint32_t)j, z);
    float4 *dst = reinterpret_cast<float4 *>(zr + ((size_t)j * N + k) * 12);
    dst[0] = make_float4(z[0], z[1], z[2], z[3]);
    dst[1] = make_float4(z[4], z[5], z[6], z[7]);
    dst[2] = make_float4(z[8], z[9], z[10], z[11]);
  }
  if (tab.write_q && j0 == 0) d.q[k] = draw_q(d, r, k);
}

// ---------------------------------------------------------------------------
// Workgroup reductions (wave64 DPP adds, then LDS across waves)
// ---------------------------------------------------------------------------
// Uniform value of lane l (a scalar read, no LDS traffic).
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// v moved by the DPP control CTRL; lanes outside the row/bank masks, and
// lanes whose source lies outside their row, read zero.
template <int CTRL, int RM, int BM>
__device__ __forceinline__ float dpp_z(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RM, BM, true));
}
template <int CTRL, int RM, int BM>
__device__ __forceinline__ double dpp_z(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, RM, BM, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, RM, BM, true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over the 64 lanes, in every lane.  Within each row of 16 lanes, lane i
// gathers x[i-3..i] (row shifts 1, 2, 3), then the partial sums of lanes
// i-4 and i-8 (banks 1-3, then 2-3), so lane 15 of a row holds the row's
// sum; row broadcasts add row 0 into row 1 and row 2 into row 3 (lane 15),
// then lane 31 into rows 2 and 3: lane 63 holds the total, read as a
// scalar.  A fixed tree, so the result is deterministic.
template <typename V>
__device__ __forceinline__ V wave_sum(V x) {
  V v = x + dpp_z<0x111, 0xF, 0xF>(x);   // row_shr:1
  v = v + dpp_z<0x112, 0xF, 0xF>(x);     // row_shr:2 (of x)
  v = v + dpp_z<0x113, 0xF, 0xF>(x);     // row_shr:3 (of x)
  v = v + dpp_z<0x114, 0xF, 0xE>(v);     // row_shr:4, banks 1-3
  v = v + dpp_z<0x118, 0xF, 0xC>(v);     // row_shr:8, banks 2-3
  v = v + dpp_z<0x142, 0xA, 0xF>(v);     // row_bcast:15, rows 1 and 3
  v = v + dpp_z<0x143, 0xC, 0xF>(v);     // row_bcast:31, rows 2 and 3
  return read_lane(v, 63);
}

// Wave sum of v where only the lanes in `mask` (a ballot, uniform) may be
// non-zero: none -> 0, up to 8 lanes -> their values added in lane order
// through scalar reads, else the shuffle tree.  Deterministic: the path
// depends on the data alone.
template <typename V>
__device__ __forceinline__ V wave_sum_sparse(V v, uint64_t mask) {
  if (mask == 0) return V(0);
  if (__popcll(mask) <= 8) {
    V acc = V(0);
    while (mask) {
      const int l = __ffsll((long long)mask) - 1;
      acc += read_lane(v, l);
      mask &= mask - 1;
    }
    return acc;
  }
  return wave_sum(v);
}

// v of lane (this lane XOR m), through the LDS crossbar (no LDS storage).
__device__ __forceinline__ double lane_xor(double v, int m) {
  const int addr = (((int)threadIdx.x & 63) ^ m) << 2;
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Wave sums of 24 values at once, written to out[0..23] (by the lanes
// whose index is a multiple of 8).  Three halving exchanges first: across
// lanes l and l ^ m (m = 32, 16, 8) the lane whose bit m is clear keeps the
// lower half of its values and adds its partner's lower half, the other the
// upper half -- so each exchange adds half the values and moves each once --
// leaving lane l three partial sums of values 12 b5 + 6 b4 + 3 b3 + {0, 1,
// 2} (b the bits of l) over its group of 8 lanes; then three plain XOR
// steps complete them.  A fixed order, so the result is deterministic.
__device__ __forceinline__ void wave_sum24(const double (&v)[24], double *out) {
  const int lane = threadIdx.x & 63;
  double a[12], b[6], c[3];
  const bool u32 = (lane & 32) != 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const double keep = u32 ? v[12 + i] : v[i], send = u32 ? v[i] : v[12 + i];
    a[i] = keep + lane_xor(send, 32);
  }
  const bool u16 = (lane & 16) != 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const double keep = u16 ? a[6 + i] : a[i], send = u16 ? a[i] : a[6 + i];
    b[i] = keep + lane_xor(send, 16);
  }
  const bool u8 = (lane & 8) != 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double keep = u8 ? b[3 + i] : b[i], send = u8 ? b[i] : b[3 + i];
    c[i] = keep + lane_xor(send, 8);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    c[i] += lane_xor(c[i], 4);
    c[i] += lane_xor(c[i], 2);
    c[i] += lane_xor(c[i], 1);
  }
  if ((lane & 7) == 0) {
    const int base = (u32 ? 12 : 0) + (u16 ? 6 : 0) + (u8 ? 3 : 0);
#pragma unroll
    for (int i = 0; i < 3; ++i) out[base + i] = c[i];
  }
}

// (cost, index) minimum with the lowest index winning ties
template <typename T>
__device__ __forceinline__ void argmin_combine(T &v, int &k, T v2, int k2) {
  if (v2 < v || (v2 == v && k2 < k)) {
    v = v2;
    k = k2;
  }
}

// Ordering keys of costs (>= 0 or +inf): the bit patterns, in the width of
// the working precision.
__device__ __forceinline__ uint32_t key_bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint64_t key_bits(double v) { return (uint64_t)__double_as_longlong(v); }
__device__ __forceinline__ int top_bit(uint32_t v) { return 31 - __builtin_clz(v); }
__device__ __forceinline__ int top_bit(uint64_t v) { return 63 - __builtin_clzll(v); }

template <int CTRL, int RM, int BM>
__device__ __forceinline__ uint32_t dpp_zu(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, RM, BM, true);
}
template <int CTRL, int RM, int BM>
__device__ __forceinline__ uint64_t dpp_zu(uint64_t v) {
  const uint32_t lo = dpp_zu<CTRL, RM, BM>((uint32_t)v);
  const uint32_t hi = dpp_zu<CTRL, RM, BM>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t read_lane_u32(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// Inclusive prefix sum over the 64 lanes: the DPP tree of wave_sum with
// every lane's partial kept (lane i ends with x[0] + ... + x[i]).
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
  uint32_t v = x + dpp_zu<0x111, 0xF, 0xF>(x);
  v += dpp_zu<0x112, 0xF, 0xF>(x);
  v += dpp_zu<0x113, 0xF, 0xF>(x);
  v += dpp_zu<0x114, 0xF, 0xE>(v);
  v += dpp_zu<0x118, 0xF, 0xC>(v);
  v += dpp_zu<0x142, 0xA, 0xF>(v);
  v += dpp_zu<0x143, 0xC, 0xF>(v);
  return v;
}

// Largest unsigned value over the 64 lanes, in every lane (the same tree;
// zero, the identity, fills lanes outside a move's reach).
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
  uint64_t v = umax64(x, dpp_zu<0x111, 0xF, 0xF>(x));
  v = umax64(v, dpp_zu<0x112, 0xF, 0xF>(x));
  v = umax64(v, dpp_zu<0x113, 0xF, 0xF>(x));
  v = umax64(v, dpp_zu<0x114, 0xF, 0xE>(v));
  v = umax64(v, dpp_zu<0x118, 0xF, 0xC>(v));
  v = umax64(v, dpp_zu<0x142, 0xA, 0xF>(v));
  v = umax64(v, dpp_zu<0x143, 0xC, 0xF>(v));
  const uint32_t lo = read_lane_u32((uint32_t)v, 63), hi = read_lane_u32((uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

// Workgroup maxima of two unsigned values (one barrier; `red` is used by
// this call alone).
__device__ __forceinline__ void block_max2_u64(uint64_t a, uint64_t b, uint64_t (*red)[2],
                                               uint64_t &ra, uint64_t &rb) {
  a = wave_max_u64(a);
  b = wave_max_u64(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
    red[wid][0] = a;
    red[wid][1] = b;
  }
  __syncthreads();
  ra = 0;
  rb = 0;
  for (int i = 0; i < nw; ++i) {
    ra = umax64(ra, red[i][0]);
    rb = umax64(rb, red[i][1]);
  }
}

// Lowest (cost, index) over the workgroup, lowest index on ties, from each
// thread's own minimum; costs are >= 0 or +inf, so their bit patterns order
// like the values.  FP32: key and index packed into one word (one barrier);
// FP64: the key, then the index among the threads that hold it (two).
template <typename T>
__device__ __forceinline__ void block_argmin_packed(T &v, int &k, uint64_t (*red_a)[2],
                                                    uint64_t (*red_b)[2]) {
  uint64_t ra, unused;
  if constexpr (sizeof(T) == 4) {
    block_max2_u64(~(((uint64_t)key_bits(v) << 32) | (uint32_t)k), 0, red_a, ra, unused);
    v = __uint_as_float((uint32_t)(~ra >> 32));
    k = (int)(uint32_t)~ra;
  } else {
    block_max2_u64(~key_bits(v), 0, red_a, ra, unused);
    const uint64_t kmin = ~ra;
    uint64_t rk;
    block_max2_u64(key_bits(v) == kmin ? ~(uint64_t)(uint32_t)k : 0, 0, red_b, rk, unused);
    v = __longlong_as_double((long long)kmin);
    k = (int)(uint32_t)~rk;
  }
}

// ---------------------------------------------------------------------------
// Rollout
// ---------------------------------------------------------------------------
// FP32 sine and cosine: Cody-Waite reduction by pi/2 (three-part constant,
// fused multiply-adds) to |r| <= pi/4, Taylor polynomials through r^9 / r^10
// (truncation below 4e-9), quadrant by rotation.  Accurate to a few ulp for
// |x| up to ~1e4 rad; beyond that the result stays bounded.  (The
// transcendental unit's sine and cosine are about twice as fast here, but
// their error, injected at every step, costs an order of magnitude in the
// agreement of FP32 rollout costs with the FP64 oracle.)
__device__ __forceinline__ void sincos_t(float x, float *s, float *c) {
  const float n = __builtin_rintf(x * 0x1.45f306p-1f);
  float r = __builtin_fmaf(-n, 0x1.921fb6p+0f, x);
  r = __builtin_fmaf(-n, -0x1.777a5cp-25f, r);
  r = __builtin_fmaf(-n, -0x1.0p-49f, r);
  const float r2 = r * r;
  float ps = __builtin_fmaf(r2, 0x1.71de3ap-19f, -0x1.a01a02p-13f);
  ps = __builtin_fmaf(r2, ps, 0x1.111112p-7f);
  ps = __builtin_fmaf(r2, ps, -0x1.555556p-3f);
  const float sn = __builtin_fmaf(r * r2, ps, r);
  float pc = __builtin_fmaf(r2, -0x1.27e4fcp-22f, 0x1.a01a02p-16f);
  pc = __builtin_fmaf(r2, pc, -0x1.6c16c2p-10f);
  pc = __builtin_fmaf(r2, pc, 0x1.555556p-5f);
  pc = __builtin_fmaf(r2, pc, -0.5f);
  const float cs = __builtin_fmaf(r2, pc, 1.0f);
  const int q = (int)n;
  const bool swap = (q & 1) != 0;
  const float ss = swap ? cs : sn, cc = swap ? sn : cs;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}
__device__ __forceinline__ void sincos_t(double x, double *s, double *c) { sincos(x, s, c); }

// The same sine and cosine for |x| <= pi/4 (strictly: |x 2/pi| <= 1/2, where
// the reduction above picks n = 0 and leaves r = x): the polynomials alone,
// bit for bit what sincos_t returns there.
__device__ __forceinline__ bool sincos_small_arg(float x) {
  return __builtin_fabsf(x * 0x1.45f306p-1f) <= 0.5f;
}
__device__ __forceinline__ void sincos_small(float r, float *s, float *c) {
  const float r2 = r * r;
  float ps = __builtin_fmaf(r2, 0x1.71de3ap-19f, -0x1.a01a02p-13f);
  ps = __builtin_fmaf(r2, ps, 0x1.111112p-7f);
  ps = __builtin_fmaf(r2, ps, -0x1.555556p-3f);
  *s = __builtin_fmaf(r * r2, ps, r);
  float pc = __builtin_fmaf(r2, -0x1.27e4fcp-22f, 0x1.a01a02p-16f);
  pc = __builtin_fmaf(r2, pc, -0x1.6c16c2p-10f);
  pc = __builtin_fmaf(r2, pc, 0x1.555556p-5f);
  pc = __builtin_fmaf(r2, pc, -0.5f);
  *c = __builtin_fmaf(r2, pc, 1.0f);
}
// Attitude sine and cosine of one angle: where every active lane of the wave
// has a small angle (a wave-uniform branch) the reduction and quadrant steps
// are skipped.
__device__ __forceinline__ void sincos_wave(float x, float *s, float *c) {
  if (__all(sincos_small_arg(x))) sincos_small(x, s, c);
  else sincos_t(x, s, c);
}
__device__ __forceinline__ void sincos_wave(double x, double *s, double *c) { sincos_t(x, s, c); }
__device__ __forceinline__ float sqrt_t(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / __builtin_sqrt(x); }
__device__ __forceinline__ bool finite_t(float x) { return __builtin_isfinite(x); }
__device__ __forceinline__ bool finite_t(double x) { return __builtin_isfinite(x); }
__device__ __forceinline__ float exp_t(float x) { return expf(x); }
__device__ __forceinline__ double exp_t(double x) { return exp(x); }
template <typename T> __device__ __forceinline__ T inf_t();
template <> __device__ __forceinline__ float inf_t<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double inf_t<double>() { return __builtin_huge_val(); }

// The mean that iteration r samples around, row j, dimension c: the
// iteration's input buffer, read one step later when it still holds the
// previous tick's mean (the warm-start shift): row j + 1 of per-step GRFs,
// or the spline of the knots evaluated one step later; the last row hover.
template <typename T>
__device__ __forceinline__ const T *mean_in(const TickDesc &d, int r) {
  return reinterpret_cast<const T *>(d.mu_buf[(d.mu_par0 + r) & 1]);
}
template <typename T>
__device__ __forceinline__ T *mean_out(const TickDesc &d, int r) {
  return reinterpret_cast<T *>(d.mu_buf[(d.mu_par0 + r + 1) & 1]);
}
// Knot j < M - 1 of the shifted spline mean: an FP64 sum in a fixed order
// without contraction (the host's export of the state forms the same sum).
template <typename T>
__device__ __forceinline__ double shifted_knot(const TickDesc &d, const T *m, int j, int c) {
#pragma clang fp contract(off)
  const int b = d.sh_b[j];
  double v = d.sh_w[4 * j] * (double)m[b * 12 + c];
  for (int t = 1; t < 4; ++t)
    if (b + t < d.M) v = v + d.sh_w[4 * j + t] * (double)m[(b + t) * 12 + c];
  return v;
}
template <typename T>
__device__ __forceinline__ T mean_at(const TickDesc &d, const T *m, int r, int j, int c) {
  if (r == 0 && d.shift0) {
    if (j + 1 >= d.M) return (c % 3 == 2) ? (T)(0.5 * d.mass * d.gravity) : T(0);
    if (!d.spline) return m[(j + 1) * 12 + c];
    return (T)shifted_knot(d, m, j, c);
  }
  return m[j * 12 + c];
}

// Friction cone: f_z >= 0 and the tangential part scaled radially onto
// |f_t| <= mu f_z.
template <typename T>
__device__ __forceinline__ void friction_clip(T &fx, T &fy, T &fz, T mu) {
  fz = fz > T(0) ? fz : T(0);
  const T t2 = fx * fx + fy * fy;
  const T lim = mu * fz;
  const T s = (t2 > lim * lim) ? lim * rsqrt_t(t2) : T(1);
  fx *= s;
  fy *= s;
}

// Loop-invariant parameters of one controller in the working precision.
// The tracking cost sum_i Q_i (x_i - x^r_i)^2 is formed as sum_i e_i^2 with
// e_i = sqrt(Q_i) x_i - sqrt(Q_i) x^r_i (one FMA per error); the reference
// position moves with the reference velocity, so its scaled form is
// sq_pr + t sq_vr.  The Euler update's dt is folded into the constants that
// scale the accelerations (dt / m, dt / I).
template <typename T>
struct RollConst {
  T dt, g, mg, mu_f, rho, f_nom, dt_m, dt_g;
  T I[3], dt_iI[3], hip[12], Rw[12], vr[3], inv_g;
  T sq[12], sq_pr[3], sq_vr[3], sq_yaw;
  T sigma0;
};

template <typename T>
__device__ __forceinline__ void load_const(const TickDesc &d, RollConst<T> &c) {
  c.dt = (T)d.dt; c.g = (T)d.gravity; c.mg = (T)(d.mass * d.gravity);
  c.mu_f = (T)d.mu_fric; c.rho = (T)d.rho; c.f_nom = (T)d.f_nominal; c.inv_g = (T)d.inv_g;
  c.dt_m = (T)(d.dt * d.inv_mass);
  c.dt_g = (T)(d.dt * d.gravity);
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    c.hip[i] = (T)d.hip[i]; c.Rw[i] = (T)d.Rw[i]; c.sq[i] = (T)__builtin_sqrt(d.Q[i]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    c.I[i] = (T)d.inertia[i]; c.dt_iI[i] = (T)(d.dt * d.inv_inertia[i]);
    c.vr[i] = (T)d.v_ref[i];
    c.sq_pr[i] = (T)(__builtin_sqrt(d.Q[i]) * d.p_ref0[i]);
    c.sq_vr[i] = (T)(__builtin_sqrt(d.Q[i]) * d.v_ref[i]);
  }
  c.sq_yaw = (T)(__builtin_sqrt(d.Q[5]) * d.yaw_ref);
  c.sigma0 = (T)d.sigma0;
}

// The policy's sample theta = mu + sigma z as one fused multiply-add, in
// every rollout form (so that forms that pick their operands differently
// still round alike).
template <typename T>
__device__ __forceinline__ T theta_of(T mu, T sig, T z) {
  if constexpr (sizeof(T) == 8) return __builtin_fma(sig, z, mu);
  else return __builtin_fmaf(sig, z, mu);
}

// One lane per sample.  The block stages the controller's mean (and the elite
// std of later iterations) in LDS once; each step reads them as broadcasts,
// and the noise of step j+1 is requested while step j computes.
// GEN (FP32, per-step GRFs): the rollout makes its sample's noise itself,
// with the noise kernel's own Philox counter and transform.  GEN 1: all of
// row j at step j, stored for the update instead of read: the same values,
// one launch and a 48-B read per rollout-step fewer.  GEN 2 (stance-pair
// form): only the Gaussians of the stance diagonal's six GRF components --
// three of the row's six Box-Muller pairs, from two or three of its Philox
// calls -- and nothing stored; the update makes the rows of the samples it
// weighs (MPPI) or chooses (elite, best sample) itself (noise_row, the same
// values).
template <typename T, int BLOCK, int UNROLL, bool INL, bool SPL, bool PAIR, int GEN = 0>
__global__ void __launch_bounds__(BLOCK) k_rollout(LaunchTab tab, TickDesc inl) {
  extern __shared__ __align__(16) unsigned char roll_lds[];
  const int b = blockIdx.x;
  const int it = stage_item<INL>(tab.roll_start, tab.n, b);
  const TickDesc &d = INL ? inline_desc() : tab.desc[tab.item[it]];
  const int N = d.N, H = d.H, M = d.M;
  T *s_mu = reinterpret_cast<T *>(roll_lds);
  T *s_sig = s_mu + (size_t)tab.max_rows * 12;
  T *s_spw = s_sig + (size_t)tab.max_rows * 12;                        // SPL: [H][4]
  int *s_spb = reinterpret_cast<int *>(s_spw + (size_t)tab.max_h * 4);  // SPL: [H]
  const bool elite_sigma = (d.method == 1) && (tab.r > 0);
  // PAIR: per stance slot (pair A = legs 0, 3; pair B = legs 1, 2) the leg's
  // hip offset and GRF weights, [pair][slot][hx, hy, hz, Rx, Ry, Rz, -, -]; a
  // lane reads its pair's two rows with one address (selecting between two
  // uniform constants per lane would take register moves for every value)
  __shared__ __align__(16) T s_pair[2][2][8];
  {
    const T *mu = mean_in<T>(d, tab.r);
    for (int i = threadIdx.x; i < M * 12; i += BLOCK) {
      s_mu[i] = mean_at<T>(d, mu, tab.r, i / 12, i % 12);
      s_sig[i] = elite_sigma ? (T)d.sigma[i] : (T)d.sigma0;
    }
    if constexpr (SPL) {
      for (int i = threadIdx.x; i < H * 4; i += BLOCK) s_spw[i] = (T)d.sp_w[i];
      for (int i = threadIdx.x; i < H; i += BLOCK) s_spb[i] = d.sp_b[i];
    }
    if constexpr (PAIR) {
      for (int i = threadIdx.x; i < 32; i += BLOCK) {
        const int pr = i >> 4, sl = (i >> 3) & 1, e = i & 7;
        const int leg = pr == 0 ? (sl == 0 ? 0 : 3) : (sl == 0 ? 1 : 2);
        s_pair[pr][sl][e] = e < 3 ? (T)d.hip[3 * leg + e] : e < 6 ? (T)d.Rw[3 * leg + e - 3] : T(0);
      }
    }
  }
  __syncthreads();
  const int k = (b - stage_start<INL>(tab.roll_start, it)) * BLOCK + (int)threadIdx.x;
  if (k >= N) return;

  RollConst<T> c;
  load_const<T>(d, c);
  const T mg2 = c.mg * T(0.5), mg3 = c.mg / T(3), mg4 = c.mg * T(0.25);
  const uint32_t q = draw_q(d, tab.r, k);
  d.q[k] = q;
  const double fkd = (double)q * d.inv_q_scale;
  const T fk = (T)fkd;
  const T half_tst = (q > 0u) ? (T)(d.half_duty / fkd) : T(0);
  const uint32_t duty_q = d.duty_q;
  const bool duty_full = d.duty_full != 0;
  const bool friction = d.friction_on != 0;

  T x[12], pf[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) { x[i] = (T)d.x0[i]; pf[i] = (T)d.foot[i]; }
  uint32_t ph[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) ph[l] = d.phase_robot + d.phase_offset[l];
  // a leg touches down where it is in stance and was not at the previous
  // step; starting from "in stance" keeps the first step's feet where the
  // tick put them
  bool prev[4] = {true, true, true, true};
  T J = T(0), Jc = T(0), tj = T(0);

  static_assert(!GEN || (!SPL && sizeof(T) == 4), "noise made in the rollout: FP32 per-step GRFs");
  static_assert(GEN != 2 || PAIR, "stance legs' noise only: stance-pair form");
  const float4 *zp =
      reinterpret_cast<const float4 *>(d.z + (size_t)tab.r * d.z_iter_stride + (size_t)k * 12);
  const size_t zstride = (size_t)N * 3;  // float4 per row
  float4 z0, z1, z2;
  if constexpr (!GEN) {
    z0 = zp[0];
    z1 = zp[1];
    z2 = zp[2];
  }
  const float4 *zq = zp + (H > 1 ? zstride : 0);  // row min(j + 1, H - 1)
  // GEN: the noise counter words that do not change along the rollout
  const uint32_t key0 = (uint32_t)d.seed, key1 = (uint32_t)(d.seed >> 32);
  const uint32_t rw = (uint32_t)tab.r << 8, tick = d.tick;
  // spline: the sample's knots wb .. wb + 3 (theta = mu + sigma z), and the
  // noise of knot wb + 4 loaded ahead
  T win[4][12];
  int wb = 0;
  if constexpr (SPL) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), bq = a, cq = a;
      if (w < M) { a = zp[w * zstride]; bq = zp[w * zstride + 1]; cq = zp[w * zstride + 2]; }
      const float zw[12] = {a.x, a.y, a.z, a.w, bq.x, bq.y, bq.z, bq.w, cq.x, cq.y, cq.z, cq.w};
#pragma unroll
      for (int i = 0; i < 12; ++i)
        win[w][i] = (w < M) ? theta_of<T>(s_mu[w * 12 + i], s_sig[w * 12 + i], (T)zw[i]) : T(0);
    }
    if (4 < M) { z0 = zp[4 * zstride]; z1 = zp[4 * zstride + 1]; z2 = zp[4 * zstride + 2]; }
  }

  // The step loop, in two forms.  The general one handles every gait: all
  // four legs' forces are formed, clipped and masked by stance.  The
  // stance-pair one (PAIR) serves the diagonal trot with duty factor 1/2,
  // where at every step exactly one pair -- legs {0, 3} while leg 0's phase
  // is below D_q, legs {1, 2} otherwise -- is in stance: it forms the
  // forces, footholds, costs and torques of those two legs only.  The swing
  // legs' terms in the general form are exact zeros added in leg order, so
  // both forms compute the same sums.
  auto steps = [&](auto pair_tag) {
    constexpr bool PAIRS = decltype(pair_tag)::value;
    // PAIR: world feet of the stance pair's lower- and higher-indexed legs,
    // starting from the tick's footholds of the pair in stance at step 0
    const uint32_t phA0 = ph[0];
    bool sA_prev = duty_full || (phA0 < duty_q);
    T f0[3], f1[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      f0[i] = sA_prev ? pf[i] : pf[3 + i];
      f1[i] = sA_prev ? pf[9 + i] : pf[6 + i];
    }
#pragma unroll UNROLL
    for (int j = 0; j < H; ++j) {
      T u[12];
      T ulo[3], uhi[3];  // GEN 2: the stance legs' GRFs (lower-, higher-indexed leg)
      if constexpr (SPL) {
        while (s_spb[j] != wb) {  // uniform: the window moves on knot by knot
          const int p = wb + 4;
          const float zw[12] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w,
                                z2.x, z2.y, z2.z, z2.w};
#pragma unroll
          for (int i = 0; i < 12; ++i) {
            win[0][i] = win[1][i];
            win[1][i] = win[2][i];
            win[2][i] = win[3][i];
            win[3][i] = (p < M) ? theta_of<T>(s_mu[p * 12 + i], s_sig[p * 12 + i], (T)zw[i]) : T(0);
          }
          ++wb;
          if (wb + 4 < M) {
            const float4 *zn = zp + (size_t)(wb + 4) * zstride;
            z0 = zn[0]; z1 = zn[1]; z2 = zn[2];
          }
        }
        const T w0 = s_spw[4 * j], w1 = s_spw[4 * j + 1], w2 = s_spw[4 * j + 2], w3 = s_spw[4 * j + 3];
#pragma unroll
        for (int i = 0; i < 12; ++i)
          u[i] = w0 * win[0][i] + w1 * win[1][i] + w2 * win[2][i] + w3 * win[3][i];
      } else if constexpr (GEN == 2) {
        // the stance diagonal's three Box-Muller pairs: pair A (legs 0, 3)
        // pairs 0, 1 (call 0) and 2 (words 0, 1 of call 1); pair B (legs 1,
        // 2) pairs 3 (words 2, 3 of call 1), 4 and 5 (call 2).  Every lane
        // makes call 1 and one more call, 0 or 2 by its pair (the counter is
        // per lane, so a wave that mixes the pairs still makes two calls);
        // slot s gives the lower-indexed stance leg's component s and the
        // other leg's.
        const bool sA = duty_full || (ph[0] < duty_q);
        uint32_t m0 = (uint32_t)k, m1 = (uint32_t)j, m2 = tick, m3 = rw | 1u;
        philox4x32_10(m0, m1, m2, m3, key0, key1);
        uint32_t o0 = (uint32_t)k, o1 = (uint32_t)j, o2 = tick, o3 = rw | (sA ? 0u : 2u);
        philox4x32_10(o0, o1, o2, o3, key0, key1);
        const float2 g0 = gauss_pair(sA ? o0 : m2, sA ? o1 : m3);  // pair 0 | 3: x forces
        const float2 g1 = gauss_pair(sA ? o2 : o0, sA ? o3 : o1);  // pair 1 | 4: y forces
        const float2 g2 = gauss_pair(sA ? m0 : o2, sA ? m1 : o3);  // pair 2 | 5: z forces
        const float zl[3] = {g0.x, g1.x, g2.x};
        const float zh[3] = {g0.y, g1.y, g2.y};
        const int bl = j * 12 + (sA ? 0 : 3), bh = j * 12 + (sA ? 9 : 6);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          ulo[i] = theta_of<T>(s_mu[bl + i], s_sig[bl + i], (T)zl[i]);
          uhi[i] = theta_of<T>(s_mu[bh + i], s_sig[bh + i], (T)zh[i]);
        }
      } else if constexpr (GEN == 1) {
        float zz[12];
        noise_row(key0, key1, rw, tick, (uint32_t)k, (uint32_t)j, zz);
        float4 *dst = const_cast<float4 *>(zp) + (size_t)j * zstride;
        dst[0] = make_float4(zz[0], zz[1], zz[2], zz[3]);
        dst[1] = make_float4(zz[4], zz[5], zz[6], zz[7]);
        dst[2] = make_float4(zz[8], zz[9], zz[10], zz[11]);
        const T *muj = s_mu + j * 12;
        const T *sgj = s_sig + j * 12;
#pragma unroll
        for (int i = 0; i < 12; ++i) u[i] = theta_of<T>(muj[i], sgj[i], (T)zz[i]);
      } else {
        const float zz[12] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w,
                              z2.x, z2.y, z2.z, z2.w};
        const T *muj = s_mu + j * 12;
        const T *sgj = s_sig + j * 12;
#pragma unroll
        for (int i = 0; i < 12; ++i) u[i] = theta_of<T>(muj[i], sgj[i], (T)zz[i]);
        // the next step's noise (the last step reads its own row again), into
        // the registers this step's noise has just left
        z0 = zq[0]; z1 = zq[1]; z2 = zq[2];
        zq += (j + 2 < H) ? zstride : 0;
      }
      // attitude
      T sr, cr, sp, cp, sy, cy;
      sincos_wave(x[3], &sr, &cr);
      sincos_wave(x[4], &sp, &cp);
      sincos_wave(x[5], &sy, &cy);
      const T spsr = sp * sr, spcr = sp * cr;
      const T R00 = cy * cp, R01 = cy * spsr - sy * cr, R02 = cy * spcr + sy * sr;
      const T R10 = sy * cp, R11 = sy * spsr + cy * cr, R12 = sy * spcr - cy * sr;
      const T R20 = -sp, R21 = cp * sr, R22 = cp * cr;
      // capture-point base of Eq. (2) for legs touching down at this step
      const T zc = x[2] > T(0) ? x[2] : T(0);
      const T cap = sqrt_t(zc * c.inv_g);
      const T bx = x[0] + half_tst * c.vr[0] + cap * (x[6] - c.vr[0]);
      const T by = x[1] + half_tst * c.vr[1] + cap * (x[7] - c.vr[1]);
      // tracking part of the stage cost (Sec. V); each form adds its legs'
      // GRF terms to it in leg order
      auto tracking = [&]() -> T {
        const T e0 = c.sq[0] * x[0] - (c.sq_pr[0] + tj * c.sq_vr[0]);
        const T e1 = c.sq[1] * x[1] - (c.sq_pr[1] + tj * c.sq_vr[1]);
        const T e2 = c.sq[2] * x[2] - (c.sq_pr[2] + tj * c.sq_vr[2]);
        const T e3 = c.sq[3] * x[3], e4 = c.sq[4] * x[4], e5 = c.sq[5] * x[5] - c.sq_yaw;
        const T e6 = c.sq[6] * x[6] - c.sq_vr[0], e7 = c.sq[7] * x[7] - c.sq_vr[1];
        const T e8 = c.sq[8] * x[8] - c.sq_vr[2];
        const T e9 = c.sq[9] * x[9], e10 = c.sq[10] * x[10], e11 = c.sq[11] * x[11];
        return e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3 + e4 * e4 + e5 * e5 + e6 * e6 + e7 * e7 +
               e8 * e8 + e9 * e9 + e10 * e10 + e11 * e11;
      };
      T stage;
      T Fx = T(0), Fy = T(0), Fz = T(0), tx = T(0), ty = T(0), tz = T(0);
      if constexpr (PAIRS) {
        const bool sA = duty_full || (ph[0] < duty_q);
        const bool td = sA != sA_prev;  // the pair in stance has just touched down
        sA_prev = sA;
        // the stance legs: 0 and 3 (pair A) or 1 and 2 (pair B), in leg order
        const T *pc = &s_pair[sA ? 0 : 1][0][0];
        T v0[3], v1[3], h0[3], h1[3], r0[3], r1[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          if constexpr (GEN == 2) {
            v0[i] = ulo[i];
            v1[i] = uhi[i];
          } else {
            v0[i] = sA ? u[i] : u[3 + i];
            v1[i] = sA ? u[9 + i] : u[6 + i];
          }
          h0[i] = pc[i];
          r0[i] = pc[3 + i];
          h1[i] = pc[8 + i];
          r1[i] = pc[11 + i];
        }
        {  // footholds of Eq. (2) at touchdown
          const T n0x = bx + R00 * h0[0] + R01 * h0[1] + R02 * h0[2];
          const T n0y = by + R10 * h0[0] + R11 * h0[1] + R12 * h0[2];
          const T n1x = bx + R00 * h1[0] + R01 * h1[1] + R02 * h1[2];
          const T n1y = by + R10 * h1[0] + R11 * h1[1] + R12 * h1[2];
          f0[0] = td ? n0x : f0[0];
          f0[1] = td ? n0y : f0[1];
          f0[2] = td ? T(0) : f0[2];
          f1[0] = td ? n1x : f1[0];
          f1[1] = td ? n1y : f1[1];
          f1[2] = td ? T(0) : f1[2];
        }
        if (friction) {
          friction_clip<T>(v0[0], v0[1], v0[2], c.mu_f);
          friction_clip<T>(v1[0], v1[1], v1[2], c.mu_f);
        }
        // two legs in stance: each carries half the weight in u^r
        stage = tracking();
        {
          const T ez0 = v0[2] - mg2, ez1 = v1[2] - mg2;
          stage += r0[0] * v0[0] * v0[0] + r0[1] * v0[1] * v0[1] + r0[2] * ez0 * ez0;
          stage += r1[0] * v1[0] * v1[0] + r1[1] * v1[1] * v1[1] + r1[2] * ez1 * ez1;
        }
        {
          const T lx = f0[0] - x[0], ly = f0[1] - x[1], lz = f0[2] - x[2];
          Fx += v0[0]; Fy += v0[1]; Fz += v0[2];
          tx += ly * v0[2] - lz * v0[1];
          ty += lz * v0[0] - lx * v0[2];
          tz += lx * v0[1] - ly * v0[0];
        }
        {
          const T lx = f1[0] - x[0], ly = f1[1] - x[1], lz = f1[2] - x[2];
          Fx += v1[0]; Fy += v1[1]; Fz += v1[2];
          tx += ly * v1[2] - lz * v1[1];
          ty += lz * v1[0] - lx * v1[2];
          tz += lx * v1[1] - ly * v1[0];
        }
      } else {
        // contact schedule
        bool st[4];
        int nst = 0;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          st[l] = duty_full || (ph[l] < duty_q);
          nst += st[l] ? 1 : 0;
        }
        // footholds of the legs touching down at this step (Eq. (2))
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const bool td = st[l] && !prev[l];
          const T hx = c.hip[3 * l], hy = c.hip[3 * l + 1], hz = c.hip[3 * l + 2];
          const T nx = bx + R00 * hx + R01 * hy + R02 * hz;
          const T ny = by + R10 * hx + R11 * hy + R12 * hz;
          pf[3 * l + 0] = td ? nx : pf[3 * l + 0];
          pf[3 * l + 1] = td ? ny : pf[3 * l + 1];
          pf[3 * l + 2] = td ? T(0) : pf[3 * l + 2];
          prev[l] = st[l];
        }
        // policy: theta = mu + sigma z (per step, or the spline of the knots),
        // clipped to the cone, masked by stance
        if (friction) {
#pragma unroll
          for (int l = 0; l < 4; ++l) friction_clip<T>(u[3 * l], u[3 * l + 1], u[3 * l + 2], c.mu_f);
        }
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          u[3 * l] = st[l] ? u[3 * l] : T(0);
          u[3 * l + 1] = st[l] ? u[3 * l + 1] : T(0);
          u[3 * l + 2] = st[l] ? u[3 * l + 2] : T(0);
        }
        T share = c.mg;  // m g / n_stance, selected without branches
        share = (nst >= 2) ? mg2 : share;
        share = (nst >= 3) ? mg3 : share;
        share = (nst >= 4) ? mg4 : share;
        stage = tracking();
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const T ez = u[3 * l + 2] - (st[l] ? share : T(0));
          stage += c.Rw[3 * l] * u[3 * l] * u[3 * l] + c.Rw[3 * l + 1] * u[3 * l + 1] * u[3 * l + 1] +
                   c.Rw[3 * l + 2] * ez * ez;
        }
        // SRBD derivative, Eq. (1), with world-frame lever arms to the feet
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const T lx = pf[3 * l] - x[0], ly = pf[3 * l + 1] - x[1], lz = pf[3 * l + 2] - x[2];
          const T ux = u[3 * l], uy = u[3 * l + 1], uz = u[3 * l + 2];
          Fx += ux; Fy += uy; Fz += uz;
          tx += ly * uz - lz * uy;
          ty += lz * ux - lx * uz;
          tz += lx * uy - ly * ux;
        }
      }
      {  // compensated accumulation
        const T y = stage - Jc;
        const T t = J + y;
        Jc = (t - J) - y;
        J = t;
      }
      const T tbx = R00 * tx + R10 * ty + R20 * tz;  // R^T tau_world
      const T tby = R01 * tx + R11 * ty + R21 * tz;
      const T tbz = R02 * tx + R12 * ty + R22 * tz;
      const T wx = x[9], wy = x[10], wz = x[11];
      const T Iwx = c.I[0] * wx, Iwy = c.I[1] * wy, Iwz = c.I[2] * wz;
      const T gx = wy * Iwz - wz * Iwy, gy = wz * Iwx - wx * Iwz, gz = wx * Iwy - wy * Iwx;
      const T icp = rcp_t(cp);
      const T a = sr * wy + cr * wz;
      const T dphi = wx + a * sp * icp;
      const T dth = cr * wy - sr * wz;
      const T dpsi = a * icp;
      // explicit Euler
      x[0] += c.dt * x[6];
      x[1] += c.dt * x[7];
      x[2] += c.dt * x[8];
      x[3] += c.dt * dphi;
      x[4] += c.dt * dth;
      x[5] += c.dt * dpsi;
      x[6] += c.dt_m * Fx;
      x[7] += c.dt_m * Fy;
      x[8] += c.dt_m * Fz - c.dt_g;
      x[9] += c.dt_iI[0] * (tbx - gx);
      x[10] += c.dt_iI[1] * (tby - gy);
      x[11] += c.dt_iI[2] * (tbz - gz);
      if constexpr (PAIRS) {
        ph[0] += q;
      } else {
#pragma unroll
        for (int l = 0; l < 4; ++l) ph[l] += q;
      }
      tj += c.dt;
    }
  };
  steps(std::integral_constant<bool, PAIR>{});
  const T df = fk - c.f_nom;
  J += c.rho * df * df;
  if (!(J >= T(0)) || !finite_t(J)) J = inf_t<T>();
  reinterpret_cast<T *>(d.J)[k] = J;
}

// ---------------------------------------------------------------------------
// Rollout, four lanes per sample (FP32).  Lane l of a quad owns leg l: its
// noise, policy, friction clip, foothold, force and torque, its GRF cost and
// the cost of state group l ([p, Phi, v, omega][l]).  The three attitude
// sin/cos pairs are computed by lanes 0..2 and broadcast inside the quad;
// net force and torque are quad sums (DPP).  Every lane integrates the full
// state from the same quad-uniform values, so the four copies stay
// identical.  Used when a launch has few samples: four times the waves at
// roughly half the instructions per lane-step.
// ---------------------------------------------------------------------------
// Quad permutation (every source lane lies inside the quad and quads leave
// the kernel whole, so bound_ctrl never applies; setting it lets the compiler
// fold the move into the consuming add as a DPP operand).
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float quad_sum(float v) {
  v = v + dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  return v + dpp<0x4E>(v);  // quad_perm [2,3,0,1]
}

template <int BLOCK, int UNROLL, bool INL, bool SPL>
__global__ void __launch_bounds__(BLOCK) k_rollout_quad(LaunchTab tab, TickDesc inl) {
  extern __shared__ __align__(16) unsigned char roll_lds[];
  constexpr int kPerBlock = BLOCK / 4;
  const int b = blockIdx.x;
  const int it = stage_item<INL>(tab.roll_start, tab.n, b);
  const TickDesc &d = INL ? inline_desc() : tab.desc[tab.item[it]];
  const int N = d.N, H = d.H, M = d.M;
  const bool elite_sigma = (d.method == 1) && (tab.r > 0);
  float *s_mu = reinterpret_cast<float *>(roll_lds);
  float *s_sig = s_mu + (size_t)tab.max_rows * 12;
  float *s_spw = s_sig + (size_t)tab.max_rows * 12;                     // SPL: [H][4]
  int *s_spb = reinterpret_cast<int *>(s_spw + (size_t)tab.max_h * 4);  // SPL: [H]
  {
    const float *mu = mean_in<float>(d, tab.r);
    for (int i = threadIdx.x; i < M * 12; i += BLOCK) {
      s_mu[i] = mean_at<float>(d, mu, tab.r, i / 12, i % 12);
      s_sig[i] = elite_sigma ? (float)d.sigma[i] : (float)d.sigma0;
    }
    if constexpr (SPL) {
      for (int i = threadIdx.x; i < H * 4; i += BLOCK) s_spw[i] = (float)d.sp_w[i];
      for (int i = threadIdx.x; i < H; i += BLOCK) s_spb[i] = d.sp_b[i];
    }
  }
  __syncthreads();
  const int l = threadIdx.x & 3;
  const int k = (b - stage_start<INL>(tab.roll_start, it)) * kPerBlock + (int)(threadIdx.x >> 2);
  if (k >= N) return;  // whole quads leave together

  const float dt = (float)d.dt;
  const float dt_m = (float)(d.dt * d.inv_mass), dt_g = (float)(d.dt * d.gravity);
  const float mg = (float)(d.mass * d.gravity), mu_f = (float)d.mu_fric, inv_g = (float)d.inv_g;
  const float mg2 = mg * 0.5f, mg3 = mg / 3.f, mg4 = mg * 0.25f;
  const float I0 = (float)d.inertia[0], I1 = (float)d.inertia[1], I2 = (float)d.inertia[2];
  const float dt_iI0 = (float)(d.dt * d.inv_inertia[0]), dt_iI1 = (float)(d.dt * d.inv_inertia[1]),
              dt_iI2 = (float)(d.dt * d.inv_inertia[2]);
  const float vr0 = (float)d.v_ref[0], vr1 = (float)d.v_ref[1], vr2 = (float)d.v_ref[2];
  const float hx = (float)d.hip[3 * l], hy = (float)d.hip[3 * l + 1], hz = (float)d.hip[3 * l + 2];
  const float Rw0 = (float)d.Rw[3 * l], Rw1 = (float)d.Rw[3 * l + 1], Rw2 = (float)d.Rw[3 * l + 2];
  // tracking errors of state group l scaled by sqrt(Q): e = sq x - sq x^r,
  // the reference being position (moving with v_ref), attitude (0, 0,
  // yaw_ref), velocity v_ref, angular velocity 0
  const double qa = __builtin_sqrt(d.Q[3 * l]), qb = __builtin_sqrt(d.Q[3 * l + 1]),
               qc = __builtin_sqrt(d.Q[3 * l + 2]);
  const float sqa = (float)qa, sqb = (float)qb, sqc = (float)qc;
  const float ra0 = (float)(qa * ((l == 0) ? d.p_ref0[0] : (l == 2) ? d.v_ref[0] : 0.0));
  const float ra1 = (float)(qb * ((l == 0) ? d.p_ref0[1] : (l == 2) ? d.v_ref[1] : 0.0));
  const float ra2 = (float)(qc * ((l == 0) ? d.p_ref0[2] : (l == 1) ? d.yaw_ref
                                                          : (l == 2) ? d.v_ref[2] : 0.0));
  const float rv0 = (float)(qa * ((l == 0) ? d.v_ref[0] : 0.0));
  const float rv1 = (float)(qb * ((l == 0) ? d.v_ref[1] : 0.0));
  const float rv2 = (float)(qc * ((l == 0) ? d.v_ref[2] : 0.0));
  const uint32_t q = draw_q(d, tab.r, k);
  if (l == 0) d.q[k] = q;
  const double fkd = (double)q * d.inv_q_scale;
  const float half_tst = (q > 0u) ? (float)(d.half_duty / fkd) : 0.f;
  const uint32_t duty_q = d.duty_q;
  const bool duty_full = d.duty_full != 0;
  const bool friction = d.friction_on != 0;

  float x[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) x[i] = (float)d.x0[i];
  float pfx = (float)d.foot[3 * l], pfy = (float)d.foot[3 * l + 1], pfz = (float)d.foot[3 * l + 2];
  uint32_t ph = d.phase_robot + d.phase_offset[l];
  bool prev = true;  // no touchdown at the first step (tick's footholds)
  float J = 0.f, Jc = 0.f, tj = 0.f;

  const float *zp = d.z + (size_t)tab.r * d.z_iter_stride + (size_t)k * 12 + 3 * l;
  const size_t zstride = (size_t)N * 12;
  float za = zp[0], zb = zp[1], zc = zp[2];
  const float *zq = zp + (H > 1 ? zstride : 0);  // row min(j + 1, H - 1)
  // spline: this leg's three forces at knots wb .. wb + 3, and the noise of
  // knot wb + 4 loaded ahead
  float win[4][3];
  int wb = 0;
  if constexpr (SPL) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
        win[w][i] = (w < M) ? theta_of<float>(s_mu[w * 12 + 3 * l + i], s_sig[w * 12 + 3 * l + i],
                                              zp[w * zstride + i])
                            : 0.f;
    }
    if (4 < M) { za = zp[4 * zstride]; zb = zp[4 * zstride + 1]; zc = zp[4 * zstride + 2]; }
  }

#pragma unroll UNROLL
  for (int j = 0; j < H; ++j) {
    float ux, uy, uz;
    if constexpr (SPL) {
      while (s_spb[j] != wb) {  // uniform: the window moves on knot by knot
        const int p = wb + 4, o = p * 12 + 3 * l;
        const float zn3[3] = {za, zb, zc};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          win[0][i] = win[1][i];
          win[1][i] = win[2][i];
          win[2][i] = win[3][i];
          win[3][i] = (p < M) ? theta_of<float>(s_mu[o + i], s_sig[o + i], zn3[i]) : 0.f;
        }
        ++wb;
        if (wb + 4 < M) {
          const float *zn = zp + (size_t)(wb + 4) * zstride;
          za = zn[0]; zb = zn[1]; zc = zn[2];
        }
      }
      const float w0 = s_spw[4 * j], w1 = s_spw[4 * j + 1], w2 = s_spw[4 * j + 2], w3 = s_spw[4 * j + 3];
      ux = w0 * win[0][0] + w1 * win[1][0] + w2 * win[2][0] + w3 * win[3][0];
      uy = w0 * win[0][1] + w1 * win[1][1] + w2 * win[2][1] + w3 * win[3][1];
      uz = w0 * win[0][2] + w1 * win[1][2] + w2 * win[2][2] + w3 * win[3][2];
    } else {
      const int o = j * 12 + 3 * l;
      ux = theta_of<float>(s_mu[o], s_sig[o], za);
      uy = theta_of<float>(s_mu[o + 1], s_sig[o + 1], zb);
      uz = theta_of<float>(s_mu[o + 2], s_sig[o + 2], zc);
      // the next step's noise (the last step reads its own row again)
      za = zq[0]; zb = zq[1]; zc = zq[2];
      zq += (j + 2 < H) ? zstride : 0;
    }
    const bool st = duty_full || (ph < duty_q);
    const float nst = quad_sum(st ? 1.f : 0.f);
    // attitude: lanes 0, 1, 2 take roll, pitch, yaw
    const float ang = (l == 0) ? x[3] : (l == 1) ? x[4] : x[5];
    float sv, cv;
    sincos_wave(ang, &sv, &cv);
    const float sr = dpp<0x00>(sv), cr = dpp<0x00>(cv);
    const float sp = dpp<0x55>(sv), cp = dpp<0x55>(cv);
    const float sy = dpp<0xAA>(sv), cy = dpp<0xAA>(cv);
    const float spsr = sp * sr, spcr = sp * cr;
    const float R00 = cy * cp, R01 = cy * spsr - sy * cr, R02 = cy * spcr + sy * sr;
    const float R10 = sy * cp, R11 = sy * spsr + cy * cr, R12 = sy * spcr - cy * sr;
    const float R20 = -sp, R21 = cp * sr, R22 = cp * cr;
    // foothold of this leg when it touches down (Eq. (2))
    {
      const float zcm = x[2] > 0.f ? x[2] : 0.f;
      const float cap = sqrt_t(zcm * inv_g);
      const bool td = st && !prev;
      const float nx = x[0] + half_tst * vr0 + cap * (x[6] - vr0) + R00 * hx + R01 * hy + R02 * hz;
      const float ny = x[1] + half_tst * vr1 + cap * (x[7] - vr1) + R10 * hx + R11 * hy + R12 * hz;
      pfx = td ? nx : pfx;
      pfy = td ? ny : pfy;
      pfz = td ? 0.f : pfz;
      prev = st;
    }
    // policy of this leg
    if (friction) friction_clip<float>(ux, uy, uz, mu_f);
    ux = st ? ux : 0.f;
    uy = st ? uy : 0.f;
    uz = st ? uz : 0.f;
    // stage cost: this leg's GRF error and state group l's tracking error
    float share = mg;  // m g / n_stance, selected without branches
    share = (nst > 1.5f) ? mg2 : share;
    share = (nst > 2.5f) ? mg3 : share;
    share = (nst > 3.5f) ? mg4 : share;
    const float ez = uz - (st ? share : 0.f);
    const float ga = (l == 0) ? x[0] : (l == 1) ? x[3] : (l == 2) ? x[6] : x[9];
    const float gb = (l == 0) ? x[1] : (l == 1) ? x[4] : (l == 2) ? x[7] : x[10];
    const float gc = (l == 0) ? x[2] : (l == 1) ? x[5] : (l == 2) ? x[8] : x[11];
    const float e0 = sqa * ga - (ra0 + tj * rv0), e1 = sqb * gb - (ra1 + tj * rv1);
    const float e2 = sqc * gc - (ra2 + tj * rv2);
    const float stage = e0 * e0 + e1 * e1 + e2 * e2 + Rw0 * ux * ux + Rw1 * uy * uy +
                        Rw2 * ez * ez;
    {
      const float y = stage - Jc;
      const float t = J + y;
      Jc = (t - J) - y;
      J = t;
    }
    // net force and torque about the CoM (world frame)
    const float lx = pfx - x[0], ly = pfy - x[1], lz = pfz - x[2];
    const float Fx = quad_sum(ux), Fy = quad_sum(uy), Fz = quad_sum(uz);
    const float tx = quad_sum(ly * uz - lz * uy);
    const float ty = quad_sum(lz * ux - lx * uz);
    const float tz = quad_sum(lx * uy - ly * ux);
    const float tbx = R00 * tx + R10 * ty + R20 * tz;
    const float tby = R01 * tx + R11 * ty + R21 * tz;
    const float tbz = R02 * tx + R12 * ty + R22 * tz;
    const float wx = x[9], wy = x[10], wz = x[11];
    const float Iwx = I0 * wx, Iwy = I1 * wy, Iwz = I2 * wz;
    const float gx = wy * Iwz - wz * Iwy, gy = wz * Iwx - wx * Iwz, gz = wx * Iwy - wy * Iwx;
    const float icp = rcp_t(cp);
    const float a = sr * wy + cr * wz;
    const float dphi = wx + a * sp * icp;
    const float dth = cr * wy - sr * wz;
    const float dpsi = a * icp;
    x[0] += dt * x[6];
    x[1] += dt * x[7];
    x[2] += dt * x[8];
    x[3] += dt * dphi;
    x[4] += dt * dth;
    x[5] += dt * dpsi;
    x[6] += dt_m * Fx;
    x[7] += dt_m * Fy;
    x[8] += dt_m * Fz - dt_g;
    x[9] += dt_iI0 * (tbx - gx);
    x[10] += dt_iI1 * (tby - gy);
    x[11] += dt_iI2 * (tbz - gz);
    ph += q;
    tj += dt;
  }
  float Jt = quad_sum(J);
  const float df = (float)fkd - (float)d.f_nominal;
  Jt += (float)d.rho * df * df;
  if (!(Jt >= 0.f) || !finite_t(Jt)) Jt = inf_t<float>();
  if (l == 0) reinterpret_cast<float *>(d.J)[k] = Jt;
}

// ---------------------------------------------------------------------------
// Select (elite and best-sample updates): one workgroup per controller.
// Thread t owns the contiguous samples [t P, (t+1) P), P = max(16,
// ceil(N / 1024)), the first 16 held in registers (the rest read again from
// memory).  Output: the chosen samples in index order (act, actw) -- the K_e
// elites or the best sample -- and per-iteration scalars.  MPPI controllers
// form their weights inside k_update_mppi and leave this stage at once.
//
// Every workgroup-wide step costs one barrier: wave results go through DPP
// (no LDS permutes) and each step has LDS slots of its own, so no barrier
// guards a slot's reuse.  Steps: lowest (cost, index) and highest cost key;
// per radix digit a histogram pass; one prefix scan of the below-threshold
// and tie counts; one sum of the elite frequency moments.
// ---------------------------------------------------------------------------
constexpr int kSelPer = 16;
// Radix histograms: kSelCopies copies of 256 bins, copy = lane mod
// kSelCopies, rows padded to kHistStride words so that one bin of different
// copies sits in different LDS banks.  Lanes that share a digit then add into
// different words: a skewed cost distribution (most samples in one bin, as
// the +inf costs of diverged rollouts are) no longer serialises a wave's
// atomics on one address.
constexpr int kSelCopies = 16;
constexpr int kHistStride = 257;
static_assert(kSelBlock == 4 * 256, "the histogram reduction gives each bin one quad of threads");

// Index of the wave's lowest (cost, index), lowest index on ties, from each
// lane's own minimum (every lane gets it; no barrier).  A wave whose lanes
// hold no sample returns the empty index 0x7fffffff.
template <typename T>
__device__ __forceinline__ int wave_argmin_index(T v, int k) {
  if constexpr (sizeof(T) == 4) {
    return (int)(uint32_t)~wave_max_u64(~(((uint64_t)key_bits(v) << 32) | (uint32_t)k));
  } else {
    const uint64_t kmin = ~wave_max_u64(~key_bits(v));
    return (int)(uint32_t)~wave_max_u64(key_bits(v) == kmin ? ~(uint64_t)(uint32_t)k : 0);
  }
}

// Exclusive workgroup prefixes of two counts and their totals (one barrier).
__device__ __forceinline__ void block_excl_scan2(uint32_t a, uint32_t b, uint2 *red,
                                                 uint32_t &a_before, uint32_t &b_before,
                                                 uint32_t &a_tot, uint32_t &b_tot) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint32_t ia = wave_incl_scan_u32(a), ib = wave_incl_scan_u32(b);
  if (lane == 63) red[wid] = make_uint2(ia, ib);
  __syncthreads();
  a_before = ia - a;
  b_before = ib - b;
  a_tot = 0;
  b_tot = 0;
  for (int i = 0; i < nw; ++i) {
    const uint2 c = red[i];
    a_before += (i < wid) ? c.x : 0u;
    b_before += (i < wid) ? c.y : 0u;
    a_tot += c.x;
    b_tot += c.y;
  }
}

// Workgroup sums of two FP64 values, waves added in order (one barrier).
__device__ __forceinline__ void block_sum2(double &a, double &b, double2 *red) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) red[wid] = make_double2(a, b);
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int i = 0; i < nw; ++i) {
    a += red[i].x;
    b += red[i].y;
  }
}

__device__ __forceinline__ float key_value(uint32_t k, float) { return __uint_as_float(k); }
__device__ __forceinline__ double key_value(uint64_t k, double) {
  return __longlong_as_double((long long)k);
}

template <typename T, bool INL>
__global__ void __launch_bounds__(kSelBlock) k_select(LaunchTab tab, TickDesc inl) {
  const TickDesc &d = INL ? inline_desc() : tab.desc[tab.item[blockIdx.x]];
  if (d.method == 0) return;  // MPPI: see k_update_mppi
  const int N = d.N, tid = threadIdx.x, lane = tid & 63;
  const T *Jg = reinterpret_cast<const T *>(d.J);
  T *actw = reinterpret_cast<T *>(d.w);
  uint32_t *act = d.act;
  const int r = tab.r;
  using K = decltype(key_bits(T(0)));
  __shared__ uint32_t hist[kSelCopies * kHistStride];
  __shared__ __align__(16) uint32_t bin_tot[256];  // the bin totals of a radix pass
  __shared__ uint64_t red_min[kSelBlock / 64][2];
  __shared__ uint64_t red_idx[kSelBlock / 64][2];
  __shared__ uint2 red_scan[kSelBlock / 64];
  __shared__ double2 red_sum[kSelBlock / 64];

  for (int i = tid; i < kSelCopies * kHistStride; i += kSelBlock) hist[i] = 0u;

  // thread t owns samples [t P, t P + P), P = max(kSelPer, ceil(N / 1024))
  const int per0 = (N + kSelBlock - 1) / kSelBlock;
  const int per = per0 > kSelPer ? per0 : kSelPer;
  const int k0 = tid * per;
  const int kend = (k0 + per < N) ? k0 + per : N;  // may be <= k0 for idle threads
  // costs (and, for the elite update, phase increments) of this thread's
  // first kSelPer samples in registers (FP64 controllers read the increments
  // from memory: their costs already take twice the registers).  A whole
  // slice in range is read with 16-byte loads: one wave instruction then
  // covers 1 KB, where one element per lane would touch 64 cache lines to
  // use 4 bytes of each, sixteen times over (the single workgroup's memory
  // pipeline, not the latency, bounded that phase).
  constexpr bool kQReg = sizeof(T) == 4;
  T Jr[kSelPer];
  uint32_t Qr[kQReg ? kSelPer : 1];
  const bool want_q = d.method == 1;
  if (per == kSelPer && k0 + kSelPer <= N) {
    const uint4 *src = reinterpret_cast<const uint4 *>(Jg + k0);
    constexpr int kVec = kSelPer * (int)sizeof(T) / 16;
#pragma unroll
    for (int v = 0; v < kVec; ++v) {
      const uint4 w = src[v];
      const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
      if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) Jr[4 * v + e] = __uint_as_float(ww[e]);
      } else {
#pragma unroll
        for (int e = 0; e < 2; ++e)
          Jr[2 * v + e] = __longlong_as_double((long long)(((uint64_t)ww[2 * e + 1] << 32) | ww[2 * e]));
      }
    }
    if (kQReg && want_q) {
      const uint4 *qs = reinterpret_cast<const uint4 *>(d.q + k0);
#pragma unroll
      for (int v = 0; v < kSelPer / 4; ++v) {
        const uint4 w = qs[v];
        Qr[kQReg ? 4 * v : 0] = w.x;
        Qr[kQReg ? 4 * v + 1 : 0] = w.y;
        Qr[kQReg ? 4 * v + 2 : 0] = w.z;
        Qr[kQReg ? 4 * v + 3 : 0] = w.w;
      }
    } else if (kQReg) {
#pragma unroll
      for (int i = 0; i < kSelPer; ++i) Qr[kQReg ? i : 0] = 0u;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kSelPer; ++i) {
      const int kc = k0 + i < N ? k0 + i : N - 1;
      const T jv = Jg[kc];
      Jr[i] = (k0 + i < kend) ? jv : inf_t<T>();
      if (kQReg) {
        const uint32_t qq = d.q[kc];
        Qr[kQReg ? i : 0] = (want_q && k0 + i < kend) ? qq : 0u;
      }
    }
  }
  // SEL_FOR(...): visit this thread's samples in index order with the cost
  // in `cv`, the phase increment in `qv` (elite update only) and the local
  // position in `i` (registers first, then memory)
#define SEL_FOR(...)                                                   \
  _Pragma("unroll") for (int i = 0; i < kSelPer; ++i) {                \
    if (i < per && k0 + i < kend) {                                    \
      const T cv = Jr[i];                                              \
      const uint32_t qv = kQReg ? Qr[kQReg ? i : 0]                    \
                                : (want_q ? d.q[k0 + i] : 0u);         \
      (void)qv;                                                        \
      __VA_ARGS__                                                      \
    }                                                                  \
  }                                                                    \
  for (int i = kSelPer; i < per && k0 + i < kend; ++i) {               \
    const T cv = Jg[k0 + i];                                           \
    const uint32_t qv = want_q ? d.q[k0 + i] : 0u;                     \
    (void)qv;                                                          \
    __VA_ARGS__                                                        \
  }

  if (d.dbg_J) {
    for (int k = tid; k < N; k += kSelBlock) {
      d.dbg_J[(size_t)r * N + k] = (double)Jg[k];
      d.dbg_q[(size_t)r * N + k] = d.q[k];
    }
  }
  // Costs are >= 0 or +inf, so their bit patterns order like the values.
  // Lowest (cost, index), lowest index on ties, and the highest key, as
  // maxima of complemented keys: FP32 keys pack with the index into one
  // 64-bit word; FP64 keys take a second step for the index.
  uint64_t m_lo = 0, m_hi = 0;
  SEL_FOR(
    const K key = key_bits(cv);
    m_hi = umax64(m_hi, (uint64_t)key);
    if constexpr (sizeof(K) == 4) {
      m_lo = umax64(m_lo, ~(((uint64_t)key << 32) | (uint32_t)(k0 + i)));
    } else {
      m_lo = umax64(m_lo, ~(uint64_t)key);
    })
  uint64_t r_lo, r_hi;
  block_max2_u64(m_lo, m_hi, red_min, r_lo, r_hi);
  K kmin;
  int bk;
  if constexpr (sizeof(K) == 4) {
    kmin = (K)(~r_lo >> 32);
    bk = (int)(uint32_t)~r_lo;
  } else {
    kmin = (K)~r_lo;
    uint64_t m_k = 0;
    SEL_FOR(if (key_bits(cv) == kmin) m_k = umax64(m_k, ~(uint64_t)(uint32_t)(k0 + i));)
    uint64_t r_k, unused;
    block_max2_u64(m_k, 0, red_idx, r_k, unused);
    bk = (int)(uint32_t)~r_k;
  }
  const K kmax = (K)r_hi;
  const T bv = key_value(kmin, T(0));
  const double cur_mf = (r == 0) ? d.ctl[0] : d.it[IT_MUF];
  const double cur_sf = (r == 0) ? d.sigma_f0 : d.it[IT_SIGF];
  const double prev_flags = (r == 0) ? 0.0 : d.it[IT_FLAGS];
  const bool skip = !finite_t(bv);

  double omega = 0.0, fnew = cur_mf, mf_next = cur_mf, sf_next = cur_sf;
  uint32_t nact = 0;
  if (skip) {
    nact = 0;
  } else if (d.method == 2) {  // naive: the best sample
    if (tid == 0) {
      act[0] = (uint32_t)bk;
      actw[0] = T(1);
    }
    nact = 1;
    omega = 1.0;
    fnew = (double)d.q[bk] * d.inv_q_scale;
    mf_next = fnew;
  } else {  // elite: the K_e smallest (cost, index) by radix selection
    // Every key shares the bits above the highest bit in which the lowest
    // and the highest key differ: the digits start there (up to 8 bits
    // each), so no pass is spent on a digit every key shares.
    int hi = (kmin == kmax) ? -1 : top_bit((K)(kmin ^ kmax));
    const K below = hi < 0 ? K(0) : (K)((K(2) << hi) - K(1));  // bits 0..hi (wraps to all)
    K mask = (K)~below, prefix = (K)(kmin & mask);
    uint32_t rank = (uint32_t)d.Ke;
    uint32_t *my_hist = hist + (lane & (kSelCopies - 1)) * kHistStride;
    const int bin = tid >> 2, part = tid & 3;
    while (hi >= 0) {
      const int lo = hi >= 7 ? hi - 7 : 0;
      const K dmask = (K)((K(1) << (hi - lo + 1)) - K(1));
      SEL_FOR(
        const K key = key_bits(cv);
        if ((key & mask) == prefix) atomicAdd(&my_hist[(uint32_t)((key >> lo) & dmask)], 1u);)
      __syncthreads();
      // bin totals: quad (bin, part) adds copies 4 part .. 4 part + 3 and
      // clears them for the next pass
      uint32_t c = 0;
#pragma unroll
      for (int cc = 0; cc < kSelCopies / 4; ++cc) {
        uint32_t *h = &hist[(4 * part + cc) * kHistStride + bin];
        c += *h;
        *h = 0u;
      }
      c += (uint32_t)__builtin_amdgcn_mov_dpp((int)c, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
      c += (uint32_t)__builtin_amdgcn_mov_dpp((int)c, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
      if (part == 0) bin_tot[bin] = c;
      __syncthreads();
      // every wave finds the first digit whose cumulative count reaches
      // `rank` (lane l holds digits 4l .. 4l + 3); exactly one lane's range
      // (excl, incl] holds it, since the counts add up to the keys that
      // match the prefix, at least `rank` of them
      const uint32_t hh[4] = {bin_tot[4 * lane], bin_tot[4 * lane + 1], bin_tot[4 * lane + 2],
                              bin_tot[4 * lane + 3]};
      const uint32_t sum = hh[0] + hh[1] + hh[2] + hh[3];
      const uint32_t incl = wave_incl_scan_u32(sum), excl = incl - sum;
      uint32_t cum = excl, dg = 0;
      for (dg = 0; dg < 3u; ++dg) {
        if (cum + hh[dg] >= rank) break;
        cum += hh[dg];
      }
      const uint64_t owner = __ballot(excl < rank && rank <= incl);
      const int src = __ffsll((long long)owner) - 1;
      const uint32_t digit = read_lane_u32(4u * (uint32_t)lane + dg, src);
      rank = read_lane_u32(rank - cum, src);
      prefix |= (K)((K)digit << lo);
      mask |= (K)(dmask << lo);
      hi = lo - 1;
    }
    // prefix is the K_e-th smallest cost; the first `rank` ties by index are in
    const K thr = prefix;
    const uint32_t need = rank;
    uint32_t nless = 0, ntie = 0;
    SEL_FOR(
      const K key = key_bits(cv);
      nless += (key < thr) ? 1u : 0u;
      ntie += (key == thr) ? 1u : 0u;)
    uint32_t less_before, tie_before, tot_less, tot_tie;
    block_excl_scan2(nless, ntie, red_scan, less_before, tie_before, tot_less, tot_tie);
    // elites before this thread: every lower key, and the ties of lower
    // index up to `need`
    uint32_t tb = tie_before;
    uint32_t pos = less_before + (tie_before < need ? tie_before : need);
    double s1 = 0.0, s2 = 0.0;
    SEL_FOR(
      const K key = key_bits(cv);
      bool el = key < thr;
      if (key == thr) {
        el = tb < need;
        ++tb;
      }
      if (el) {
        const int k = k0 + i;
        act[pos] = (uint32_t)k;
        actw[pos] = T(1);
        ++pos;
        const double f = (double)qv * d.inv_q_scale;
        s1 += f;
        s2 += f * f;
      })
    nact = tot_less + (tot_tie < need ? tot_tie : need);
    block_sum2(s1, s2, red_sum);
    const double ke = (double)d.Ke;
    const double fm = s1 / ke;
    double fv = s2 / ke - fm * fm;
    fv = fv > 0.0 ? fv : 0.0;
    omega = ke;
    fnew = fm;
    mf_next = fm;
    const double sfl = __builtin_sqrt(fv);
    sf_next = sfl > d.sigma_min_f ? sfl : d.sigma_min_f;
  }
#undef SEL_FOR
  if (tid == 0) {
    d.it[IT_BETA] = (double)bv;
    d.it[IT_OMEGA] = omega;
    d.it[IT_BEST] = (double)bk;
    d.it[IT_FNEW] = fnew;
    d.it[IT_MUF] = mf_next;
    d.it[IT_SIGF] = sf_next;
    d.it[IT_SKIP] = skip ? 1.0 : 0.0;
    d.it[IT_FLAGS] = (double)((int)prev_flags | (skip ? 1 : 0));
    d.it[IT_NACT] = (double)nact;
  }
}

// ---------------------------------------------------------------------------
// Update: one workgroup per (controller, step j).  It reduces
// S1[c] = sum over the chosen samples of w_k z_kjc (and S2 = sum of z_kjc^2
// for the elite, whose weights are 1) and writes step j of the new mean:
//   MPPI / best sample:  mu'_jc = mu_jc + sigma0 S1 / Omega
//   elite:               mu'_jc = mu_jc + sigma_jc m,  sigma'_jc = max(sigma_jc sqrt(v), floor)
// with m = S1 / K_e, v = S2 / K_e - m^2 (FP64).  Each step is independent, so
// no workgroup waits for another; the warm-start shift is left to the next
// reader of the mean.  Step 0 of the last iteration also writes the action.
// k_update serves the elite and best-sample controllers from k_select's
// output; k_update_mppi forms the MPPI weights itself.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void contact_at(const TickDesc &d, bool st[4]) {
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const uint32_t ph = d.phase_robot + d.phase_offset[l];
    st[l] = d.duty_full ? true : (ph < d.duty_q);
  }
}

// The action record (Fig. 2: the first step of the new mean goes to the
// low-level controller): u_0 masked by the contact flags at the robot's
// phase and clipped to the friction cone, the executed frequency and its
// phase increment, the lowest cost, flags and the number of samples that
// carried weight; the record's sequence word goes last.  Also stores the
// frequency mean for the next tick.
__device__ __forceinline__ void emit_action(const TickDesc &d, const double *s_new, double f_new,
                                            double beta, double flags, double nact) {
  const double f_final = (d.freq_mode == 0) ? d.f_fixed : f_new;
  const uint32_t qf = (d.freq_mode == 0) ? d.q_fixed : q_of_freq(f_final, d.dt);
  bool st[4];
  contact_at(d, st);
  double *res = d.result;
  for (int l = 0; l < 4; ++l) {
    double fx = s_new[3 * l], fy = s_new[3 * l + 1], fz = s_new[3 * l + 2];
    if (d.friction_on) friction_clip<double>(fx, fy, fz, d.mu_fric);
    res[RES_GRF + 3 * l + 0] = st[l] ? fx : 0.0;
    res[RES_GRF + 3 * l + 1] = st[l] ? fy : 0.0;
    res[RES_GRF + 3 * l + 2] = st[l] ? fz : 0.0;
    res[RES_CONTACT + l] = st[l] ? 1.0 : 0.0;
  }
  res[RES_FREQ] = f_final;
  res[RES_Q] = (double)qf;
  res[RES_BEST] = beta;
  res[RES_FLAGS] = flags;
  res[RES_NACT] = nact;
  d.ctl[0] = f_final;
  __hip_atomic_store(reinterpret_cast<uint64_t *>(res + RES_SEQ), (uint64_t)d.tick + 1u,
                     __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename T, bool INL>
__global__ void __launch_bounds__(kUpdBlock) k_update(LaunchTab tab, TickDesc inl) {
  const int b = blockIdx.x;
  const int item = stage_item<INL>(tab.upd_start, tab.n, b);
  const TickDesc &d = INL ? inline_desc() : tab.desc[tab.item[item]];
  if (d.method == 0) return;  // MPPI: k_update_mppi
  // steps j0 .. j1 - 1, each reduced as a one-step workgroup reduces it
  const int ch = tab.upd_chunk > 1 ? tab.upd_chunk : 1;
  const int j0 = (b - stage_start<INL>(tab.upd_start, item)) * ch;
  const int j1 = j0 + ch < d.M ? j0 + ch : d.M;
  const int N = d.N, tid = threadIdx.x;
  const int r = tab.r;
  const bool elite = (d.method == 1);
  const T *actw = reinterpret_cast<const T *>(d.w);
  const uint32_t *act = d.act;
  __shared__ double lds[kUpdBlock / 64][24];
  __shared__ double s_new[12];
  const bool last_iter = (r == d.R - 1);
  for (int j = j0; j < j1; ++j) {
    // What does not depend on the select's output is read first, so that its
    // latency overlaps the gathers: this step's old mean and std.
    double m_old = 0.0, sig = 0.0;
    if (tid < 12) {
      m_old = (double)mean_at<T>(d, mean_in<T>(d, r), r, j, tid);
      sig = (elite && r > 0) ? d.sigma[j * 12 + tid] : d.sigma0;
    }
    // The chosen samples number at most K_e (elite) or one (best sample): their
    // indices are read together with the count instead of after it, clamped
    // into [0, N) so that a stale entry never leaves the noise rows, and the
    // count (zero on a skipped iteration) masks them afterwards.
    const int nmax = elite ? d.Ke : 1;
    const bool skip = d.it[IT_SKIP] != 0.0;
    const int nact = skip ? 0 : (int)d.it[IT_NACT];

    double out1[12], out2[12];
    {
      const float *zj = d.z + (size_t)r * d.z_iter_stride + (size_t)j * N * 12;
      double s1[12], s2[12];
      T f1[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) { s1[c] = 0.0; s2[c] = 0.0; f1[c] = T(0); }
      if (tab.gen_noise == 2) {
        // the rollout stored no noise: each chosen sample's row drawn again,
        // one row per thread and pass (sample a on thread a mod the block:
        // the order of the sums the gathers below keep)
        for (int a = tid; a < nact; a += kUpdBlock) {
          const uint32_t kv = act[a];
          const uint32_t k = kv < (uint32_t)N ? kv : (uint32_t)(N - 1);
          float zz[12];
          noise_row((uint32_t)d.seed, (uint32_t)(d.seed >> 32), (uint32_t)r << 8, d.tick, k,
                    (uint32_t)j, zz);
          if (elite) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
              const double zc = (double)zz[c];
              s1[c] += zc;
              s2[c] += zc * zc;
            }
          } else {
            const T wv = actw[a];
#pragma unroll
            for (int c = 0; c < 12; ++c) f1[c] += wv * (T)zz[c];
          }
        }
      } else {
        // four gathers in flight per thread: indices and weights first, then rows
        for (int a = tid; a < nmax; a += 4 * kUpdBlock) {
          uint32_t ka[4];
          T wa[4];
          bool va[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int aa = a + u * kUpdBlock;
            const int ac = aa < nmax ? aa : nmax - 1;  // always valid: loads issue together
            const uint32_t kv = act[ac];
            const T wv = actw[ac];
            va[u] = aa < nact;
            ka[u] = kv < (uint32_t)N ? kv : (uint32_t)(N - 1);
            wa[u] = va[u] ? wv : T(0);
          }
          float4 zl[4][3];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float4 *src = reinterpret_cast<const float4 *>(zj + (size_t)ka[u] * 12);
            zl[u][0] = src[0];
            zl[u][1] = src[1];
            zl[u][2] = src[2];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (!va[u]) continue;
            const float zz[12] = {zl[u][0].x, zl[u][0].y, zl[u][0].z, zl[u][0].w,
                                  zl[u][1].x, zl[u][1].y, zl[u][1].z, zl[u][1].w,
                                  zl[u][2].x, zl[u][2].y, zl[u][2].z, zl[u][2].w};
            if (elite) {
#pragma unroll
              for (int c = 0; c < 12; ++c) {
                const double zc = (double)zz[c];
                s1[c] += zc;
                s2[c] += zc * zc;
              }
            } else {
#pragma unroll
              for (int c = 0; c < 12; ++c) f1[c] += wa[u] * (T)zz[c];
            }
          }
        }
      }
      if (elite) {
        // the wave's 12 first and 12 second moments, into this wave's row
        double v[24];
#pragma unroll
        for (int c = 0; c < 12; ++c) { v[c] = s1[c]; v[12 + c] = s2[c]; }
        wave_sum24(v, lds[tid >> 6]);
      } else {
        // reduce in the working precision within the wave, FP64 across waves
#pragma unroll
        for (int c = 0; c < 12; ++c) { out1[c] = (double)wave_sum(f1[c]); out2[c] = 0.0; }
      }
    }
    const int lane = tid & 63, wid = tid >> 6;
    if (!elite && lane == 0) {
#pragma unroll
      for (int c = 0; c < 12; ++c) { lds[wid][c] = out1[c]; lds[wid][12 + c] = out2[c]; }
    }
    __syncthreads();
    if (tid < 12) {
      const int c = tid, idx = j * 12 + c;
      double S1 = 0.0, S2 = 0.0;
      for (int i = 0; i < kUpdBlock / 64; ++i) {
        S1 += lds[i][c];
        S2 += lds[i][12 + c];
      }
      double m_new = m_old;
      if (elite) {
        double sg = sig;
        if (!skip) {
          const double omega = d.it[IT_OMEGA];
          const double mz = S1 / omega;
          double vz = S2 / omega - mz * mz;
          vz = vz > 0.0 ? vz : 0.0;
          m_new = m_old + sig * mz;
          const double sn = sig * __builtin_sqrt(vz);
          sg = sn > d.sigma_min_grf ? sn : d.sigma_min_grf;
        }
        d.sigma[idx] = sg;
      } else if (!skip) {
        m_new = m_old + d.sigma0 * (S1 / d.it[IT_OMEGA]);
      }
      const T stored = (T)m_new;
      mean_out<T>(d, r)[idx] = stored;
      if (j == 0) s_new[c] = (double)stored;
      if (last_iter && d.dbg_mean) d.dbg_mean[idx] = (double)stored;
    }
    __syncthreads();  // the next step reuses lds
  }
  if (!(last_iter && j0 == 0)) return;
  if (tid == 0)
    emit_action(d, s_new, d.it[IT_FNEW], d.it[IT_BETA], d.it[IT_FLAGS], d.it[IT_NACT]);
}

// MPPI update (Alg. 4) with the weighting fused in: every workgroup of a
// controller forms beta = min J (lowest index on ties), w_k = exp((beta -
// J_k) / lambda) in the working precision, Omega = sum w_k and the weighted
// frequency sum in FP64, in the same order, and reduces S1 over the samples
// whose weight does not underflow.  Thread t visits samples t, t + B, ...
// (coalesced cost reads and noise-row gathers).  Step 0 also leaves the
// per-iteration scalars (next iteration's frequency mean) and, in the last
// iteration, the action.
constexpr int kMppiPer = 16;

// Sample k's share of the fused MPPI sums: weight w = exp((beta - J) / lambda)
// in the working precision and, when it does not underflow, the weighted
// noise row (already requested when k is its wave's lowest cost, kw), the
// FP64 normaliser and frequency sums and the count of weighted samples.

// MPPI update (Alg. 4), one 1024-thread workgroup per controller: the
// lowest cost beta, the weights w_k = exp((beta - J_k) / lambda), the FP64
// normaliser Omega and frequency moment, then every row of the new mean,
// mu'_j = mu_j + sigma sum_k w_k z_kj / Omega.  Usually few weights do not
// underflow: their samples are listed in LDS in increasing k and each
// (row, dimension) output sums its list terms in FP64 in that order.  With
// more than kListCap of them, or N above the register-held kPer per thread,
// each row is reduced over all samples instead (per-thread partial sums in
// the working precision, wave sums, FP64 across waves).  Either way the
// result depends only on the controller's own data, not on the batch.
constexpr int kListCap = 2048;

// Noise row j of sample k made again and stored where the rollout would have
// stored it (z of iteration r: [M][N][12]).
__device__ __forceinline__ void make_noise_row(const TickDesc &d, int r, uint32_t k, uint32_t j,
                                               const float *zr) {
  float z[12];
  noise_row((uint32_t)d.seed, (uint32_t)(d.seed >> 32), (uint32_t)r << 8, d.tick, k, j, z);
  float4 *dst = reinterpret_cast<float4 *>(const_cast<float *>(zr) + ((size_t)j * d.N + k) * 12);
  dst[0] = make_float4(z[0], z[1], z[2], z[3]);
  dst[1] = make_float4(z[4], z[5], z[6], z[7]);
  dst[2] = make_float4(z[8], z[9], z[10], z[11]);
}

template <typename T, bool INL>
__global__ void __launch_bounds__(kMppiBlock) k_update_mppi(LaunchTab tab, TickDesc inl) {
  const TickDesc &d = INL ? inline_desc() : tab.desc[tab.item[blockIdx.x]];
  if (d.method != 0) return;  // elite / best sample: k_select + k_update
  const int N = d.N, M = d.M, tid = threadIdx.x, r = tab.r;
  constexpr int kW = kMppiBlock / 64;
  // the first kPer costs of each thread are held in registers (independent
  // loads, one memory latency): 16 in FP32, 2 in FP64, which keeps the FP64
  // form within a 1024-thread workgroup's 128 registers; beyond that (N
  // above kPer * kMppiBlock) they are read again from memory, in the same
  // order
  constexpr int kPer = sizeof(T) == 8 ? 2 : kMppiPer;
  __shared__ double lds[kW][16];
  __shared__ uint64_t red_a[kW][2], red_b[kW][2];
  __shared__ uint32_t s_pre[kPer][kW];  // list position of each (slot, wave)'s first entry
  __shared__ uint32_t s_total;
  __shared__ uint32_t s_k[kListCap];
  __shared__ T s_w[kListCap];
  __shared__ double s_new[12];
  const T *Jg = reinterpret_cast<const T *>(d.J);
  const bool last_iter = (r == d.R - 1);
  const double cur_mf = (r == 0) ? d.ctl[0] : d.it[IT_MUF];
  const double cur_sf = (r == 0) ? d.sigma_f0 : d.it[IT_SIGF];
  const double prev_flags = (r == 0) ? 0.0 : d.it[IT_FLAGS];
  const T *mu_in = mean_in<T>(d, r);
  T *mu_out = mean_out<T>(d, r);
  const float *zr = d.z + (size_t)r * d.z_iter_stride;

  T Jr[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int k = tid + i * kMppiBlock;
    const T jv = Jg[k < N ? k : N - 1];  // always valid: the loads issue together
    Jr[i] = (k < N) ? jv : inf_t<T>();
  }
  T bv = inf_t<T>();
  int bk = 0x7fffffff;
#pragma unroll
  for (int i = 0; i < kPer; ++i) argmin_combine(bv, bk, Jr[i], tid + i * kMppiBlock);
  for (int k = tid + kPer * kMppiBlock; k < N; k += kMppiBlock) argmin_combine(bv, bk, Jg[k], k);
  block_argmin_packed(bv, bk, red_a, red_b);
  const bool skip = !finite_t(bv);

  // 1/lambda in the working precision, kept finite: at a lambda whose
  // reciprocal overflows FP32 the best sample's (beta - J) il stays
  // 0 * finite = 0 (weight 1) rather than 0 * inf = NaN, and every other
  // weight underflows to 0 -- the argmin limit of Alg. 4
  const double ild = d.inv_lambda;
  const T il = (T)(ild < (double)std::numeric_limits<T>::max() ? ild
                                                                : (double)std::numeric_limits<T>::max());
  // weights of this thread's samples; a bit per register-held cost marks
  // those that do not underflow (their weights are formed again where
  // needed: the same values); FP64 normaliser and frequency moment
  uint32_t wmask = 0u;
  double sw = 0.0, swf = 0.0, cnt = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int k = tid + i * kMppiBlock;
    const T wk = (!skip && k < N) ? exp_t((bv - Jr[i]) * il) : T(0);
    if (wk != T(0)) {
      wmask |= 1u << i;
      cnt += 1.0;
      sw += (double)wk;
      swf += (double)wk * ((double)d.q[k] * d.inv_q_scale);
    }
  }
  if (!skip)
    for (int k = tid + kPer * kMppiBlock; k < N; k += kMppiBlock) {
      const T wk = exp_t((bv - Jg[k]) * il);
      if (wk != T(0)) {
        cnt += 1.0;
        sw += (double)wk;
        swf += (double)wk * ((double)d.q[k] * d.inv_q_scale);
      }
    }
  const int lane = tid & 63, wid = tid >> 6;
  const uint64_t live = __ballot(cnt != 0.0);
  {
    const double o12 = wave_sum_sparse(sw, live);
    const double o13 = wave_sum_sparse(swf, live);
    const double o14 = wave_sum_sparse(cnt, live);
    if (lane == 0) {
      lds[wid][12] = o12;
      lds[wid][13] = o13;
      lds[wid][14] = o14;
    }
  }
  // list positions: samples in increasing k are slot-major (k = tid + i
  // 1024), so entry (slot i, wave w, lane l) goes after every entry of the
  // lower slots, of the lower waves of slot i and of the lower lanes
  const bool regs_only = N <= kPer * kMppiBlock;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const uint64_t bal = __ballot((wmask >> i) & 1u);
    if (lane == 0) s_pre[i][wid] = (uint32_t)__popcll(bal);
  }
  __syncthreads();
  if (wid == 0) {
    // exclusive scan of the kPer x kW counts, slot-major, by one wave
    constexpr int kCells = kPer * kW, kPerLane = (kCells + 63) / 64;
    uint32_t v[kPerLane], sum = 0;
#pragma unroll
    for (int e = 0; e < kPerLane; ++e) {
      const int cell = lane * kPerLane + e;
      v[e] = cell < kCells ? s_pre[cell / kW][cell % kW] : 0u;
      sum += v[e];
    }
    const uint32_t incl = wave_incl_scan_u32(sum);
    uint32_t run = incl - sum;
#pragma unroll
    for (int e = 0; e < kPerLane; ++e) {
      const int cell = lane * kPerLane + e;
      if (cell < kCells) s_pre[cell / kW][cell % kW] = run;
      run += v[e];
    }
    if (lane == 63) s_total = incl;
  }
  __syncthreads();
  const uint32_t total = s_total;
  const bool listed = regs_only && total <= (uint32_t)kListCap;
  if (listed) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const uint64_t bal = __ballot((wmask >> i) & 1u);
      if ((wmask >> i) & 1u) {
        const uint32_t pos = s_pre[i][wid] +
                             (uint32_t)__popcll(bal & ((lane ? ~0ull >> (64 - lane) : 0ull)));
        s_k[pos] = (uint32_t)(tid + i * kMppiBlock);
        s_w[pos] = exp_t((bv - Jr[i]) * il);
      }
    }
    __syncthreads();
    if (tab.gen_noise == 2) {
      // the rollout stored no noise: the rows of the listed samples
      for (uint32_t e = tid; e < total * (uint32_t)M; e += kMppiBlock) {
        const uint32_t a = e / (uint32_t)M, j = e - a * (uint32_t)M;
        make_noise_row(d, r, s_k[a], j, zr);
      }
      __syncthreads();
    }
    double omega = 0.0;
    for (int i = 0; i < kW; ++i) omega += lds[i][12];
    for (int o = tid; o < M * 12; o += kMppiBlock) {
      const int j = o / 12, c = o - j * 12;
      const double m_old = (double)mean_at<T>(d, mu_in, r, j, c);
      const float *zc = zr + (size_t)j * N * 12 + c;
      double S1 = 0.0;
      for (uint32_t a = 0; a < total; ++a)
        S1 = __builtin_fma((double)s_w[a], (double)zc[(size_t)s_k[a] * 12], S1);
      const double m_new = skip ? m_old : m_old + d.sigma0 * (S1 / omega);
      const T stored = (T)m_new;
      mu_out[o] = stored;
      if (j == 0) s_new[c] = (double)stored;
      if (last_iter && d.dbg_mean) d.dbg_mean[o] = (double)stored;
    }
  } else {
    if (tab.gen_noise == 2) {
      // the rollout stored no noise and too many samples weigh for the
      // list: every row (slow, and rare where the previous tick weighed few)
      for (uint32_t e = tid; e < (uint32_t)N * (uint32_t)M; e += kMppiBlock) {
        const uint32_t j = e / (uint32_t)N, k = e - j * (uint32_t)N;
        make_noise_row(d, r, k, j, zr);
      }
      __syncthreads();
    }
    for (int j = 0; j < M; ++j) {
      const float4 *zj = reinterpret_cast<const float4 *>(zr) + (size_t)j * N * 3;
      T f1[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) f1[c] = T(0);
      // (the costs are read again from memory here: a rare path, and one
      // loop over k keeps the register count of the common path)
      if (!skip)
        for (int k = tid; k < N; k += kMppiBlock) {
          const T wk = exp_t((bv - Jg[k]) * il);
          if (wk == T(0)) continue;
          const float4 z0 = zj[(size_t)k * 3], z1 = zj[(size_t)k * 3 + 1],
                       z2 = zj[(size_t)k * 3 + 2];
          const float zz[12] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w,
                                z2.x, z2.y, z2.z, z2.w};
#pragma unroll
          for (int c = 0; c < 12; ++c) f1[c] += wk * (T)zz[c];
        }
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const double o = (double)wave_sum_sparse(f1[c], live);
        if (lane == 0) lds[wid][c] = o;
      }
      __syncthreads();
      if (tid < 12) {
        const int c = tid, idx = j * 12 + c;
        double S1 = 0.0, omega = 0.0;
        for (int i = 0; i < kW; ++i) {
          S1 += lds[i][c];
          omega += lds[i][12];
        }
        const double m_old = (double)mean_at<T>(d, mu_in, r, j, c);
        const double m_new = skip ? m_old : m_old + d.sigma0 * (S1 / omega);
        const T stored = (T)m_new;
        mu_out[idx] = stored;
        if (j == 0) s_new[c] = (double)stored;
        if (last_iter && d.dbg_mean) d.dbg_mean[idx] = (double)stored;
      }
      __syncthreads();  // the next row reuses lds[][0..11]
    }
  }
  if (d.dbg_J) {
    for (int k = tid; k < N; k += kMppiBlock) {
      d.dbg_J[(size_t)r * N + k] = (double)Jg[k];
      d.dbg_q[(size_t)r * N + k] = d.q[k];
    }
  }
  __syncthreads();
  if (tid == 0) {
    double omega = 0.0, sf = 0.0, nact = 0.0;
    for (int i = 0; i < kW; ++i) {
      omega += lds[i][12];
      sf += lds[i][13];
      nact += lds[i][14];
    }
    const double fnew = skip ? cur_mf : sf / omega;
    const double flags = (double)((int)prev_flags | (skip ? 1 : 0));
    d.it[IT_BETA] = (double)bv;
    d.it[IT_OMEGA] = omega;
    d.it[IT_BEST] = (double)bk;
    d.it[IT_FNEW] = fnew;
    d.it[IT_MUF] = fnew;
    d.it[IT_SIGF] = cur_sf;
    d.it[IT_SKIP] = skip ? 1.0 : 0.0;
    d.it[IT_FLAGS] = flags;
    d.it[IT_NACT] = nact;
    if (last_iter) emit_action(d, s_new, fnew, (double)bv, flags, nact);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called by the runtime)
// ---------------------------------------------------------------------------
// timing: 0 none; 1 two events around the rollout stage (ev[0], ev[1]);
// 2 five events around the four stages (ev[0..4]).
// One rollout launch; with e0 (and e1) the events take the kernel's own
// start and end times (the dispatch carries them), so the measured duration
// is the kernel's and not that of two separate event commands around it.
template <typename K>
static void launch_timed(K kernel, dim3 g, dim3 b, size_t lds, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1, const LaunchTab &tab, const TickDesc &inl) {
  if (e0) hipExtLaunchKernelGGL(kernel, g, b, (uint32_t)lds, s, e0, e1, 0, tab, inl);
  else hipLaunchKernelGGL(kernel, g, b, lds, s, tab, inl);
}

template <bool INL, bool SPL, bool PAIR>
static hipError_t launch_one_lane(const LaunchTab &tab, const TickDesc &inl, int precision,
                                  size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 rg(tab.total_roll);
  if (precision == 1) {
    launch_timed(k_rollout<double, 64, 1, INL, SPL, PAIR>, rg, dim3(64), lds, s, e0, e1, tab, inl);
    return hipSuccess;
  }
  if constexpr (!SPL) {
    if (tab.gen_noise == 2) {  // stance legs' noise only: stance-pair form, 256 lanes
      if constexpr (PAIR) {
        if (tab.roll_block != 256) return hipErrorInvalidValue;
        launch_timed(k_rollout<float, 256, 1, INL, false, true, 2>, rg, dim3(256), lds, s, e0, e1, tab, inl);
        return hipSuccess;
      }
      return hipErrorInvalidValue;
    }
    if (tab.gen_noise) {  // the rollout makes the noise (one-row loops only)
      switch (tab.roll_block) {
        case 64: launch_timed(k_rollout<float, 64, 1, INL, false, PAIR, 1>, rg, dim3(64), lds, s, e0, e1, tab, inl); break;
        case 128: launch_timed(k_rollout<float, 128, 1, INL, false, PAIR, 1>, rg, dim3(128), lds, s, e0, e1, tab, inl); break;
        case 256: launch_timed(k_rollout<float, 256, 1, INL, false, PAIR, 1>, rg, dim3(256), lds, s, e0, e1, tab, inl); break;
        default: return hipErrorInvalidValue;
      }
      return hipSuccess;
    }
  }
  switch (tab.roll_block * 4 + tab.unroll) {
    case 64 * 4 + 1: launch_timed(k_rollout<float, 64, 1, INL, SPL, PAIR>, rg, dim3(64), lds, s, e0, e1, tab, inl); break;
    case 128 * 4 + 1: launch_timed(k_rollout<float, 128, 1, INL, SPL, PAIR>, rg, dim3(128), lds, s, e0, e1, tab, inl); break;
    case 256 * 4 + 1: launch_timed(k_rollout<float, 256, 1, INL, SPL, PAIR>, rg, dim3(256), lds, s, e0, e1, tab, inl); break;
    case 64 * 4 + 2:
      if (SPL) return hipErrorInvalidValue;
      launch_timed(k_rollout<float, 64, 2, INL, false, PAIR>, rg, dim3(64), lds, s, e0, e1, tab, inl);
      break;
    case 128 * 4 + 2:
      if (SPL) return hipErrorInvalidValue;
      launch_timed(k_rollout<float, 128, 2, INL, false, PAIR>, rg, dim3(128), lds, s, e0, e1, tab, inl);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipSuccess;
}

template <bool INL, bool SPL>
static hipError_t launch_rollout_form(const LaunchTab &tab, const TickDesc &inl, int precision,
                                      size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 rg(tab.total_roll);
  if (precision == 1 || tab.lanes != 4)
    return tab.pairs ? launch_one_lane<INL, SPL, true>(tab, inl, precision, lds, s, e0, e1)
                     : launch_one_lane<INL, SPL, false>(tab, inl, precision, lds, s, e0, e1);
  if (tab.lanes == 4) {
    switch (tab.roll_block * 4 + tab.unroll) {
      case 64 * 4 + 1: launch_timed(k_rollout_quad<64, 1, INL, SPL>, rg, dim3(64), lds, s, e0, e1, tab, inl); break;
      case 128 * 4 + 1: launch_timed(k_rollout_quad<128, 1, INL, SPL>, rg, dim3(128), lds, s, e0, e1, tab, inl); break;
      case 256 * 4 + 1: launch_timed(k_rollout_quad<256, 1, INL, SPL>, rg, dim3(256), lds, s, e0, e1, tab, inl); break;
      default: return hipErrorInvalidValue;
    }
    return hipSuccess;
  }
  return hipErrorInvalidValue;
}

template <bool INL>
static hipError_t launch_rollout(const LaunchTab &tab, const TickDesc &inl, int precision,
                                 size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return tab.spline ? launch_rollout_form<INL, true>(tab, inl, precision, lds, s, e0, e1)
                    : launch_rollout_form<INL, false>(tab, inl, precision, lds, s, e0, e1);
}

template <bool INL>
static hipError_t launch_stages(const LaunchTab &tab, const TickDesc &inl, int precision,
                                hipStream_t s, int timing, hipEvent_t *ev,
                                const std::function<hipError_t()> *after_rollout) {
  // mean and sigma [max_rows][12]; spline weights [max_h][4] and bases [max_h]
  const size_t ts = precision == 1 ? 8 : 4;
  const size_t roll_lds = (size_t)tab.max_rows * 12 * 2 * ts +
                          (tab.spline ? (size_t)tab.max_h * (4 * ts + 4) : 0);
  if (timing == 2) (void)hipEventRecord(ev[0], s);
  if (!tab.skip_noise && !tab.gen_noise)
    hipLaunchKernelGGL((k_noise<INL>), dim3(tab.total_noise * tab.r_count), dim3(kNoiseBlock), 0, s,
                       tab, inl);
  // mode 1: the rollout kernel's own start and end; mode 2: event commands
  // between all stages
  if (timing == 2) (void)hipEventRecord(ev[1], s);
  hipError_t e = launch_rollout<INL>(tab, inl, precision, roll_lds, s,
                                     timing == 1 ? ev[0] : nullptr, timing == 1 ? ev[1] : nullptr);
  if (e != hipSuccess) return e;
  // work for other streams that the host should enqueue while the rollout
  // runs rather than after the whole iteration (the next tick's noise)
  if (after_rollout && *after_rollout) {
    e = (*after_rollout)();
    if (e != hipSuccess) return e;
  }
  if (timing == 2) (void)hipEventRecord(ev[2], s);
  // elite / best-sample controllers: selection, then the update; MPPI
  // controllers: the fused update alone (each kernel skips the others' items)
  const dim3 ug(tab.total_upd);
  if (tab.n_select > 0) {
    if (precision == 1)
      hipLaunchKernelGGL((k_select<double, INL>), dim3(tab.n), dim3(kSelBlock), 0, s, tab, inl);
    else
      hipLaunchKernelGGL((k_select<float, INL>), dim3(tab.n), dim3(kSelBlock), 0, s, tab, inl);
  }
  if (timing == 2) (void)hipEventRecord(ev[3], s);
  if (tab.n_select > 0) {
    if (precision == 1)
      hipLaunchKernelGGL((k_update<double, INL>), ug, dim3(kUpdBlock), 0, s, tab, inl);
    else
      hipLaunchKernelGGL((k_update<float, INL>), ug, dim3(kUpdBlock), 0, s, tab, inl);
  }
  if (tab.n_select < tab.n) {
    if (precision == 1)
      hipLaunchKernelGGL((k_update_mppi<double, INL>), dim3(tab.n), dim3(kMppiBlock), 0, s, tab, inl);
    else
      hipLaunchKernelGGL((k_update_mppi<float, INL>), dim3(tab.n), dim3(kMppiBlock), 0, s, tab, inl);
  }
  if (timing == 2) (void)hipEventRecord(ev[4], s);
  return hipGetLastError();
}

// One iteration of every stage over the launch's controllers.  With `inl`
// non-null the launch holds exactly one controller whose descriptor travels
// in the kernel arguments.
hipError_t launch_iteration(const LaunchTab &tab, int precision, hipStream_t s, int timing,
                            hipEvent_t *ev, const TickDesc *inl,
                            const std::function<hipError_t()> *after_rollout) {
  if (tab.n == 0) return hipSuccess;
  if (inl) return launch_stages<true>(tab, *inl, precision, s, timing, ev, after_rollout);
  static const TickDesc none{};
  return launch_stages<false>(tab, none, precision, s, timing, ev, after_rollout);
}

// An empty one-workgroup dispatch carrying start/stop events: the interval
// it spans is the events' own overhead (the start marker's completion to the
// dispatch's first wave), which every event-timed launch includes once.
__global__ void k_empty() {}

hipError_t launch_empty_timed(hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  hipExtLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s, e0, e1, 0);
  return hipGetLastError();
}

// The noise stage alone (iterations tab.r .. tab.r + tab.r_count - 1), with
// the descriptor inline when `inl` is non-null.
hipError_t launch_noise_only(const LaunchTab &tab, hipStream_t s, const TickDesc *inl) {
  if (tab.n == 0) return hipSuccess;
  static const TickDesc none{};
  const dim3 g(tab.total_noise * tab.r_count);
  if (inl) hipLaunchKernelGGL((k_noise<true>), g, dim3(kNoiseBlock), 0, s, tab, *inl);
  else hipLaunchKernelGGL((k_noise<false>), g, dim3(kNoiseBlock), 0, s, tab, none);
  return hipGetLastError();
}

}  // namespace sbs
