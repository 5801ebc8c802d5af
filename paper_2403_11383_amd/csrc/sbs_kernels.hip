// sbs_kernels.hip -- gfx950 kernels of one SBS control step.
//
// Stages of one iteration (Alg. 1: sampling, evaluation, sorting, update),
// each one launch over every controller of a fused batch:
//   k_noise    counter-based Gaussian noise z[j][k][12] and gait-frequency
//              increments q[k] (Sampling)
//   k_rollout  one lane per sample: SRBD rollout of Eq. (1) with explicit
//              Euler, world-fixed footholds placed by Eq. (2) at touchdown,
//              quadratic cost of Sec. V (Alg. 2, Evaluation)
//   k_select   one workgroup per controller: lowest cost, MPPI weights with
//              an FP64 normaliser (Alg. 4), top-K_e radix selection (Alg. 1)
//              or the best sample (Alg. 3); frequency update
//   k_update   weighted sums of the noise over samples, split over
//              (step, sample chunk) workgroups; the last workgroup of a
//              controller to arrive forms the new mean (and elite std), the
//              action and the warm-started mean (Sec. III-A)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sbs_device.h"

namespace sbs {

// ---------------------------------------------------------------------------
// Noise contract: Philox4x32-10 keyed by the seed, counter (k, j, tick,
// (r << 8) | call); calls 0..2 feed GRF dims 4c..4c+3 of step j, call 3 at
// j = 0 the frequency.  Gaussians by Box-Muller on 24-bit uniforms with a
// fixed sequence of IEEE FP32 operations (no contraction), so the result is
// reproducible bit for bit on any IEEE machine.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                              uint32_t &c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ float2 gauss_pair(uint32_t w0, uint32_t w1) {
#pragma clang fp contract(off)
  const uint32_t i1 = (w0 >> 8) + 1u;   // u1 = i1 2^-24 in (0, 1]
  const uint32_t i2 = w1 >> 8;          // u2 = i2 2^-24 in [0, 1)
  int e = 31 - __clz((int)i1);
  float m = (float)i1 * __uint_as_float((uint32_t)(127 - e) << 23);  // [1, 2)
  if (m > 0x1.6a09e6p+0f) {
    m = m * 0.5f;
    e = e + 1;
  }
  const float s = (m - 1.0f) / (m + 1.0f);
  const float t = s * s;
  float p = __builtin_fmaf(t, 0x1.c71c72p-4f, 0x1.24924ap-3f);
  p = __builtin_fmaf(t, p, 0x1.99999ap-3f);
  p = __builtin_fmaf(t, p, 0x1.555556p-2f);
  const float s2 = s + s;
  const float lnm = __builtin_fmaf(s2 * t, p, s2);
  const float ke = (float)(e - 24);
  const float lnu = __builtin_fmaf(ke, 0x1.62e4p-1f, __builtin_fmaf(ke, 0x1.7f7d1cp-20f, lnm));
  const float rho = __builtin_sqrtf(-2.0f * lnu);

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
  const uint32_t quad = n & 3u;
  float c = (quad == 0u) ? cs : (quad == 1u) ? -sn : (quad == 2u) ? -cs : sn;
  float sv = (quad == 0u) ? sn : (quad == 1u) ? cs : (quad == 2u) ? -sn : -cs;
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

__device__ __forceinline__ int find_item(const int32_t *start, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(kNoiseBlock) k_noise(LaunchTab tab) {
  const int b = blockIdx.x;
  const int i = find_item(tab.noise_start, tab.n, b);
  const TickDesc &d = tab.desc[tab.item[i]];
  const int local = b - tab.noise_start[i];
  const int nkb = (d.N + kNoiseBlock - 1) / kNoiseBlock;
  const int j = local / nkb;
  const int k = (local - j * nkb) * kNoiseBlock + (int)threadIdx.x;
  if (k >= d.N) return;
  const uint32_t key0 = (uint32_t)d.seed, key1 = (uint32_t)(d.seed >> 32);
  const uint32_t rw = (uint32_t)tab.r << 8;
  float z[12];
#pragma unroll
  for (uint32_t call = 0; call < 3; ++call) {
    uint32_t c0 = (uint32_t)k, c1 = (uint32_t)j, c2 = d.tick, c3 = rw | call;
    philox4x32_10(c0, c1, c2, c3, key0, key1);
    const float2 ga = gauss_pair(c0, c1);
    const float2 gb = gauss_pair(c2, c3);
    z[4 * call + 0] = ga.x;
    z[4 * call + 1] = ga.y;
    z[4 * call + 2] = gb.x;
    z[4 * call + 3] = gb.y;
  }
  float4 *dst = reinterpret_cast<float4 *>(d.z + ((size_t)j * d.N + k) * 12);
  dst[0] = make_float4(z[0], z[1], z[2], z[3]);
  dst[1] = make_float4(z[4], z[5], z[6], z[7]);
  dst[2] = make_float4(z[8], z[9], z[10], z[11]);
  if (j == 0) {
    uint32_t q;
    if (d.freq_mode == 0) {
      q = d.q_fixed;
    } else {
      uint32_t c0 = (uint32_t)k, c1 = 0u, c2 = d.tick, c3 = rw | 3u;
      philox4x32_10(c0, c1, c2, c3, key0, key1);
      if (d.freq_mode == 1) {
        const uint64_t span = (uint64_t)(d.q_hi - d.q_lo) + 1u;
        q = d.q_lo + (uint32_t)(((uint64_t)c0 * span) >> 32);
      } else {
        const double mf = (tab.r == 0) ? d.ctl[0] : d.it[IT_MUF];
        const double sf = (tab.r == 0) ? d.sigma_f0 : d.it[IT_SIGF];
        q = freq_gaussian(mf, sf, gauss_pair(c0, c1).x, d.f_min, d.f_max, d.dt);
      }
    }
    d.q[k] = q;
  }
}

// ---------------------------------------------------------------------------
// Rollout
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_t(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_t(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ float sqrt_t(float x) { return __builtin_sqrtf(x); }
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

template <typename T>
__global__ void __launch_bounds__(kRollBlock) k_rollout(LaunchTab tab) {
  const int b = blockIdx.x;
  const int it = find_item(tab.roll_start, tab.n, b);
  const TickDesc &d = tab.desc[tab.item[it]];
  const int k = (b - tab.roll_start[it]) * kRollBlock + (int)threadIdx.x;
  if (k >= d.N) return;
  const int N = d.N, H = d.H;
  const bool elite_sigma = (d.method == 1) && (tab.r > 0);
  const T* __restrict__ mu = reinterpret_cast<const T *>(d.mu);
  const float* __restrict__ zb = d.z;

  const uint32_t q = d.q[k];
  const T fk = (T)((double)q * d.inv_q_scale);
  const T half_tst = (q > 0u) ? (T)(d.half_duty / ((double)q * d.inv_q_scale)) : T(0);
  const T dt = (T)d.dt, inv_m = (T)d.inv_mass, g = (T)d.gravity, inv_g = (T)d.inv_g;
  const T mg = (T)(d.mass * d.gravity);
  const T mu_f = (T)d.mu_fric;
  const T Ix = (T)d.inertia[0], Iy = (T)d.inertia[1], Iz = (T)d.inertia[2];
  const T iIx = (T)d.inv_inertia[0], iIy = (T)d.inv_inertia[1], iIz = (T)d.inv_inertia[2];
  const T vrx = (T)d.v_ref[0], vry = (T)d.v_ref[1], vrz = (T)d.v_ref[2];

  T x[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) x[c] = (T)d.x0[c];
  T pf[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) pf[c] = (T)d.foot[c];
  uint32_t ph[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) ph[l] = d.phase_robot + d.phase_offset[l];
  bool prev[4] = {false, false, false, false};
  T J = T(0), Jc = T(0);

  for (int j = 0; j < H; ++j) {
    // noise of (j, k): three 16-byte loads, consecutive lanes contiguous
    const float4 *src = reinterpret_cast<const float4 *>(zb + ((size_t)j * N + k) * 12);
    const float4 z0 = src[0], z1 = src[1], z2 = src[2];
    const float zz[12] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w,
                          z2.x, z2.y, z2.z, z2.w};
    // contact schedule
    bool st[4];
    int nst = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      st[l] = d.duty_full ? true : (ph[l] < d.duty_q);
      nst += st[l] ? 1 : 0;
    }
    // attitude
    T sr, cr, sp, cp, sy, cy;
    sincos_t(x[3], &sr, &cr);
    sincos_t(x[4], &sp, &cp);
    sincos_t(x[5], &sy, &cy);
    const T R00 = cy * cp, R01 = cy * sp * sr - sy * cr, R02 = cy * sp * cr + sy * sr;
    const T R10 = sy * cp, R11 = sy * sp * sr + cy * cr, R12 = sy * sp * cr - cy * sr;
    const T R20 = -sp, R21 = cp * sr, R22 = cp * cr;
    // footholds of legs touching down at this step (Eq. (2))
    {
      const T zc = x[2] > T(0) ? x[2] : T(0);
      const T cap = sqrt_t(zc * inv_g);
      const T bx = x[0] + half_tst * vrx + cap * (x[6] - vrx);
      const T by = x[1] + half_tst * vry + cap * (x[7] - vry);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const bool td = (j > 0) && st[l] && !prev[l];
        const T hx = (T)d.hip[3 * l], hy = (T)d.hip[3 * l + 1], hz = (T)d.hip[3 * l + 2];
        const T nx = bx + R00 * hx + R01 * hy + R02 * hz;
        const T ny = by + R10 * hx + R11 * hy + R12 * hz;
        pf[3 * l + 0] = td ? nx : pf[3 * l + 0];
        pf[3 * l + 1] = td ? ny : pf[3 * l + 1];
        pf[3 * l + 2] = td ? T(0) : pf[3 * l + 2];
        prev[l] = st[l];
      }
    }
    // policy: theta = mu + sigma z, masked by stance and clipped to the cone
    T u[12];
    const T *muj = mu + (size_t)j * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const T sig = elite_sigma ? (T)d.sigma[j * 12 + c] : (T)d.sigma0;
      u[c] = muj[c] + sig * (T)zz[c];
    }
    if (d.friction_on) {
#pragma unroll
      for (int l = 0; l < 4; ++l) friction_clip<T>(u[3 * l], u[3 * l + 1], u[3 * l + 2], mu_f);
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      if (!st[l]) {
        u[3 * l] = T(0);
        u[3 * l + 1] = T(0);
        u[3 * l + 2] = T(0);
      }
    }
    // stage cost (Sec. V): tracking error and GRF error to the gravity share
    const T tj = (T)((double)j * d.dt);
    const T share = mg / (T)(nst > 1 ? nst : 1);
    T xr[12];
    xr[0] = (T)d.p_ref0[0] + tj * vrx;
    xr[1] = (T)d.p_ref0[1] + tj * vry;
    xr[2] = (T)d.p_ref0[2] + tj * vrz;
    xr[3] = T(0);
    xr[4] = T(0);
    xr[5] = (T)d.yaw_ref;
    xr[6] = vrx;
    xr[7] = vry;
    xr[8] = vrz;
    xr[9] = T(0);
    xr[10] = T(0);
    xr[11] = T(0);
    T stage = T(0);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const T e = x[c] - xr[c];
      stage += (T)d.Q[c] * e * e;
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const T ex = u[3 * l], ey = u[3 * l + 1], ez = u[3 * l + 2] - (st[l] ? share : T(0));
      stage += (T)d.Rw[3 * l] * ex * ex + (T)d.Rw[3 * l + 1] * ey * ey + (T)d.Rw[3 * l + 2] * ez * ez;
    }
    {  // compensated accumulation
      const T y = stage - Jc;
      const T t = J + y;
      Jc = (t - J) - y;
      J = t;
    }
    // SRBD derivative, Eq. (1)
    T Fx = T(0), Fy = T(0), Fz = T(0), tx = T(0), ty = T(0), tz = T(0);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const T lx = pf[3 * l] - x[0], ly = pf[3 * l + 1] - x[1], lz = pf[3 * l + 2] - x[2];
      const T ux = u[3 * l], uy = u[3 * l + 1], uz = u[3 * l + 2];
      Fx += ux;
      Fy += uy;
      Fz += uz;
      tx += ly * uz - lz * uy;
      ty += lz * ux - lx * uz;
      tz += lx * uy - ly * ux;
    }
    const T tbx = R00 * tx + R10 * ty + R20 * tz;   // R^T tau_world
    const T tby = R01 * tx + R11 * ty + R21 * tz;
    const T tbz = R02 * tx + R12 * ty + R22 * tz;
    const T wx = x[9], wy = x[10], wz = x[11];
    const T Iwx = Ix * wx, Iwy = Iy * wy, Iwz = Iz * wz;
    const T gx = wy * Iwz - wz * Iwy, gy = wz * Iwx - wx * Iwz, gz = wx * Iwy - wy * Iwx;
    const T icp = rcp_t(cp);
    const T tpn = sp * icp;
    const T a = sr * wy + cr * wz;
    const T dphi = wx + a * tpn;
    const T dth = cr * wy - sr * wz;
    const T dpsi = a * icp;
    const T dvx = Fx * inv_m, dvy = Fy * inv_m, dvz = Fz * inv_m - g;
    const T dwx = (tbx - gx) * iIx, dwy = (tby - gy) * iIy, dwz = (tbz - gz) * iIz;
    // explicit Euler
    x[0] += dt * x[6];
    x[1] += dt * x[7];
    x[2] += dt * x[8];
    x[3] += dt * dphi;
    x[4] += dt * dth;
    x[5] += dt * dpsi;
    x[6] += dt * dvx;
    x[7] += dt * dvy;
    x[8] += dt * dvz;
    x[9] += dt * dwx;
    x[10] += dt * dwy;
    x[11] += dt * dwz;
#pragma unroll
    for (int l = 0; l < 4; ++l) ph[l] += q;
  }
  const T df = fk - (T)d.f_nominal;
  J += (T)d.rho * df * df;
  if (!(J >= T(0)) || !finite_t(J)) J = inf_t<T>();
  reinterpret_cast<T *>(d.J)[k] = J;
}

// ---------------------------------------------------------------------------
// Workgroup reductions (wave64 shuffles, then LDS across waves)
// ---------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename V>
__device__ V block_sum(V v, V *lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  V r = V(0);
  for (int i = 0; i < nw; ++i) r += lds[i];
  return r;
}

// (cost, index) minimum with the lowest index winning ties
template <typename T>
__device__ __forceinline__ void argmin_combine(T &v, int &k, T v2, int k2) {
  if (v2 < v || (v2 == v && k2 < k)) {
    v = v2;
    k = k2;
  }
}

template <typename T>
__device__ void block_argmin(T &v, int &k, T *lv, int *lk) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const T v2 = __shfl_xor(v, o, 64);
    const int k2 = __shfl_xor(k, o, 64);
    argmin_combine(v, k, v2, k2);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
    lv[wid] = v;
    lk[wid] = k;
  }
  __syncthreads();
  v = lv[0];
  k = lk[0];
  for (int i = 1; i < nw; ++i) argmin_combine(v, k, lv[i], lk[i]);
}

__device__ __forceinline__ uint64_t key_bits(float v) { return (uint64_t)__float_as_uint(v); }
__device__ __forceinline__ uint64_t key_bits(double v) { return (uint64_t)__double_as_longlong(v); }

// ---------------------------------------------------------------------------
// Select: one workgroup per controller
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kSelBlock) k_select(LaunchTab tab) {
  const TickDesc &d = tab.desc[tab.item[blockIdx.x]];
  const int N = d.N, tid = threadIdx.x, nt = blockDim.x;
  const T *J = reinterpret_cast<const T *>(d.J);
  T *w = reinterpret_cast<T *>(d.w);
  const int r = tab.r;
  __shared__ double lds_d[kSelBlock / 64];
  __shared__ T lds_v[kSelBlock / 64];
  __shared__ int lds_k[kSelBlock / 64];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_digit, s_rank;
  __shared__ uint32_t wave_cnt[kSelBlock / 64];

  if (d.dbg_J) {
    for (int k = tid; k < N; k += nt) {
      d.dbg_J[(size_t)r * N + k] = (double)J[k];
      d.dbg_q[(size_t)r * N + k] = d.q[k];
    }
  }
  // lowest cost and its index
  T bv = inf_t<T>();
  int bk = 0x7fffffff;
  for (int k = tid; k < N; k += nt) argmin_combine(bv, bk, J[k], k);
  block_argmin(bv, bk, lds_v, lds_k);
  const double cur_mf = (r == 0) ? d.ctl[0] : d.it[IT_MUF];
  const double cur_sf = (r == 0) ? d.sigma_f0 : d.it[IT_SIGF];
  const double prev_flags = (r == 0) ? 0.0 : d.it[IT_FLAGS];
  const bool skip = !finite_t(bv);

  double omega = 0.0, fnew = cur_mf, mf_next = cur_mf, sf_next = cur_sf;
  if (skip) {
    for (int k = tid; k < N; k += nt) w[k] = T(0);
  } else if (d.method == 0) {  // MPPI
    const T il = (T)d.inv_lambda;
    double sw = 0.0, swf = 0.0;
    for (int k = tid; k < N; k += nt) {
      const T wk = exp_t((bv - J[k]) * il);
      w[k] = wk;
      sw += (double)wk;
      swf += (double)wk * ((double)d.q[k] * d.inv_q_scale);
    }
    sw = block_sum(sw, lds_d);
    swf = block_sum(swf, lds_d);
    omega = sw;
    fnew = swf / sw;
    mf_next = fnew;
  } else if (d.method == 2) {  // naive: best sample
    for (int k = tid; k < N; k += nt) w[k] = (k == bk) ? T(1) : T(0);
    omega = 1.0;
    fnew = (double)d.q[bk] * d.inv_q_scale;
    mf_next = fnew;
  } else {  // elite: K_e smallest (cost, index) by radix selection on cost bits
    const int nbits = (int)sizeof(T) * 8;
    uint64_t prefix = 0, mask = 0;
    uint32_t rank = (uint32_t)d.Ke;
    for (int shift = nbits - 8; shift >= 0; shift -= 8) {
      for (int i = tid; i < 256; i += nt) hist[i] = 0u;
      __syncthreads();
      for (int k = tid; k < N; k += nt) {
        const uint64_t key = key_bits(J[k]);
        if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
      }
      __syncthreads();
      if (tid == 0) {
        uint32_t cum = 0, dg = 0;
        for (dg = 0; dg < 255u; ++dg) {
          if (cum + hist[dg] >= rank) break;
          cum += hist[dg];
        }
        s_digit = dg;
        s_rank = rank - cum;
      }
      __syncthreads();
      prefix |= (uint64_t)s_digit << shift;
      mask |= (uint64_t)255u << shift;
      rank = s_rank;
      __syncthreads();
    }
    // prefix is the K_e-th smallest cost; the first `rank` ties (by index)
    // are elite.
    const uint64_t thr = prefix;
    const uint32_t need = rank;
    uint32_t ties_before = 0;
    double s1 = 0.0, s2 = 0.0;
    const int lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
    for (int base = 0; base < N; base += nt) {
      const int k = base + tid;
      const uint64_t key = (k < N) ? key_bits(J[k]) : ~0ull;
      const bool tie = (k < N) && (key == thr);
      const uint64_t bal = __ballot(tie);
      const uint32_t in_wave = __popcll(bal & ((1ull << lane) - 1ull));
      __syncthreads();
      if (lane == 0) wave_cnt[wid] = __popcll(bal);
      __syncthreads();
      uint32_t before = ties_before + in_wave;
      uint32_t total = 0;
      for (int i = 0; i < nw; ++i) {
        if (i < wid) before += wave_cnt[i];
        total += wave_cnt[i];
      }
      ties_before += total;
      if (k < N) {
        const bool el = (key < thr) || (tie && before < need);
        w[k] = el ? T(1) : T(0);
        if (el) {
          const double f = (double)d.q[k] * d.inv_q_scale;
          s1 += f;
          s2 += f * f;
        }
      }
    }
    s1 = block_sum(s1, lds_d);
    s2 = block_sum(s2, lds_d);
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
  if (tid == 0) {
    d.it[IT_BETA] = (double)bv;
    d.it[IT_OMEGA] = omega;
    d.it[IT_BEST] = (double)bk;
    d.it[IT_FNEW] = fnew;
    d.it[IT_MUF] = mf_next;
    d.it[IT_SIGF] = sf_next;
    d.it[IT_SKIP] = skip ? 1.0 : 0.0;
    d.it[IT_FLAGS] = (double)((int)prev_flags | (skip ? 1 : 0));
  }
}


// ---------------------------------------------------------------------------
// Update: S1[j][d] = sum_k w_k z_kjd (and S2 = sum_k w_k z_kjd^2 for elite),
// reduced per (step, chunk) workgroup, then combined by the last workgroup of
// the controller to arrive, which writes the new mean, the elite std, the
// action and the warm-started mean.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void contact_at(const TickDesc &d, bool st[4]) {
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const uint32_t ph = d.phase_robot + d.phase_offset[l];
    st[l] = d.duty_full ? true : (ph < d.duty_q);
  }
}

template <typename T>
__global__ void __launch_bounds__(kUpdBlock) k_update(LaunchTab tab) {
  const int b = blockIdx.x;
  const int item = find_item(tab.upd_start, tab.n, b);
  const TickDesc &d = tab.desc[tab.item[item]];
  const int local = b - tab.upd_start[item];
  const int nblk = tab.upd_start[item + 1] - tab.upd_start[item];
  const int j = local / d.nchunk;
  const int ch = local - j * d.nchunk;
  const int N = d.N, H = d.H, tid = threadIdx.x;
  const int r = tab.r;
  const bool elite = (d.method == 1);
  const T *w = reinterpret_cast<const T *>(d.w);
  __shared__ double lds[kUpdBlock / 64][24];
  __shared__ int s_last;

  const int k0 = ch * kUpdChunk;
  const int k1 = (k0 + kUpdChunk < N) ? k0 + kUpdChunk : N;
  double out1[12], out2[12];
  if (elite) {
    double a1[12], a2[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) { a1[c] = 0.0; a2[c] = 0.0; }
    for (int k = k0 + tid; k < k1; k += kUpdBlock) {
      const T wk = w[k];
      if (wk != T(0)) {
        const float4 *src = reinterpret_cast<const float4 *>(d.z + ((size_t)j * N + k) * 12);
        const float4 z0 = src[0], z1 = src[1], z2 = src[2];
        const float zz[12] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w,
                              z2.x, z2.y, z2.z, z2.w};
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const double zc = (double)zz[c];
          a1[c] += zc;
          a2[c] += zc * zc;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) { out1[c] = a1[c]; out2[c] = a2[c]; }
  } else {
    T a1[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) a1[c] = T(0);
    for (int k = k0 + tid; k < k1; k += kUpdBlock) {
      const T wk = w[k];
      if (wk != T(0)) {
        const float4 *src = reinterpret_cast<const float4 *>(d.z + ((size_t)j * N + k) * 12);
        const float4 z0 = src[0], z1 = src[1], z2 = src[2];
        const float zz[12] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w,
                              z2.x, z2.y, z2.z, z2.w};
#pragma unroll
        for (int c = 0; c < 12; ++c) a1[c] += wk * (T)zz[c];
      }
    }
    // reduce in the working precision within the wave, then FP64 across
#pragma unroll
    for (int c = 0; c < 12; ++c) { out1[c] = (double)wave_sum(a1[c]); out2[c] = 0.0; }
  }
  const int lane = tid & 63, wid = tid >> 6;
  if (elite) {
#pragma unroll
    for (int c = 0; c < 12; ++c) { out1[c] = wave_sum(out1[c]); out2[c] = wave_sum(out2[c]); }
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < 12; ++c) { lds[wid][c] = out1[c]; lds[wid][12 + c] = out2[c]; }
  }
  __syncthreads();
  if (tid < 24) {
    double s = 0.0;
    for (int i = 0; i < kUpdBlock / 64; ++i) s += lds[i][tid];
    d.partial[((size_t)j * d.nchunk + ch) * 24 + tid] = s;
  }
  // arrival: the last workgroup of this controller combines
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const uint32_t old = atomicAdd(d.counter, 1u);
    s_last = (old == (uint32_t)(nblk - 1)) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();

  __shared__ double newmu[kMaxH * 12];
  const bool skip = d.it[IT_SKIP] != 0.0;
  const double omega = d.it[IT_OMEGA];
  T *mu = reinterpret_cast<T *>(d.mu);
  for (int idx = tid; idx < H * 12; idx += kUpdBlock) {
    const int jj = idx / 12, c = idx - jj * 12;
    const double m_old = (double)mu[idx];
    double m_new = m_old;
    if (!skip) {
      double s1 = 0.0, s2 = 0.0;
      for (int cc = 0; cc < d.nchunk; ++cc) {
        const double *p = d.partial + ((size_t)jj * d.nchunk + cc) * 24;
        s1 += p[c];
        s2 += p[12 + c];
      }
      if (elite) {
        const double sig = (r == 0) ? d.sigma0 : d.sigma[idx];
        const double mz = s1 / omega;
        double vz = s2 / omega - mz * mz;
        vz = vz > 0.0 ? vz : 0.0;
        m_new = m_old + sig * mz;
        const double sn = sig * __builtin_sqrt(vz);
        d.sigma[idx] = sn > d.sigma_min_grf ? sn : d.sigma_min_grf;
      } else {
        m_new = m_old + d.sigma0 * (s1 / omega);
      }
    }
    newmu[idx] = (double)(T)m_new;
  }
  if (tid == 0) *d.counter = 0u;
  __syncthreads();
  const bool last_iter = (r == d.R - 1);
  if (!last_iter) {
    for (int idx = tid; idx < H * 12; idx += kUpdBlock) mu[idx] = (T)newmu[idx];
    return;
  }
  const double hover = 0.5 * d.mass * d.gravity;
  for (int idx = tid; idx < H * 12; idx += kUpdBlock) {
    if (d.dbg_mean) d.dbg_mean[idx] = newmu[idx];
    const int jj = idx / 12, c = idx - jj * 12;
    const double v = (jj < H - 1) ? newmu[idx + 12] : ((c % 3 == 2) ? hover : 0.0);
    mu[idx] = (T)v;
  }
  if (tid == 0) {
    const double f_final = (d.freq_mode == 0) ? d.f_fixed : d.it[IT_FNEW];
    const uint32_t qf = (d.freq_mode == 0) ? d.q_fixed : q_of_freq(f_final, d.dt);
    bool st[4];
    contact_at(d, st);
    double *res = d.result;
    for (int l = 0; l < 4; ++l) {
      double fx = newmu[3 * l], fy = newmu[3 * l + 1], fz = newmu[3 * l + 2];
      if (d.friction_on) friction_clip<double>(fx, fy, fz, d.mu_fric);
      res[RES_GRF + 3 * l + 0] = st[l] ? fx : 0.0;
      res[RES_GRF + 3 * l + 1] = st[l] ? fy : 0.0;
      res[RES_GRF + 3 * l + 2] = st[l] ? fz : 0.0;
      res[RES_CONTACT + l] = st[l] ? 1.0 : 0.0;
    }
    res[RES_FREQ] = f_final;
    res[RES_Q] = (double)qf;
    res[RES_BEST] = d.it[IT_BETA];
    res[RES_FLAGS] = d.it[IT_FLAGS];
    d.ctl[0] = f_final;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called by the runtime)
// ---------------------------------------------------------------------------
hipError_t launch_iteration(const LaunchTab &tab, int precision, hipStream_t s,
                            hipEvent_t *ev /* 5 events or null */) {
  if (tab.n == 0) return hipSuccess;
  if (ev) (void)hipEventRecord(ev[0], s);
  hipLaunchKernelGGL(k_noise, dim3(tab.total_noise), dim3(kNoiseBlock), 0, s, tab);
  if (ev) (void)hipEventRecord(ev[1], s);
  if (precision == 1) {
    hipLaunchKernelGGL(k_rollout<double>, dim3(tab.total_roll), dim3(kRollBlock), 0, s, tab);
    if (ev) (void)hipEventRecord(ev[2], s);
    hipLaunchKernelGGL(k_select<double>, dim3(tab.n), dim3(kSelBlock), 0, s, tab);
    if (ev) (void)hipEventRecord(ev[3], s);
    hipLaunchKernelGGL(k_update<double>, dim3(tab.total_upd), dim3(kUpdBlock), 0, s, tab);
  } else {
    hipLaunchKernelGGL(k_rollout<float>, dim3(tab.total_roll), dim3(kRollBlock), 0, s, tab);
    if (ev) (void)hipEventRecord(ev[2], s);
    hipLaunchKernelGGL(k_select<float>, dim3(tab.n), dim3(kSelBlock), 0, s, tab);
    if (ev) (void)hipEventRecord(ev[3], s);
    hipLaunchKernelGGL(k_update<float>, dim3(tab.total_upd), dim3(kUpdBlock), 0, s, tab);
  }
  if (ev) (void)hipEventRecord(ev[4], s);
  return hipGetLastError();
}

hipError_t launch_noise_only(const LaunchTab &tab, hipStream_t s) {
  if (tab.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_noise, dim3(tab.total_noise), dim3(kNoiseBlock), 0, s, tab);
  return hipGetLastError();
}

}  // namespace sbs
