// Kino-PAX iteration kernels for gfx950 (CDNA4, wave64).
//
// The planning loop (kp_plan, Alg. 1) runs each iteration as two launches on
// one stream:
//   k_propagate  Alg. 2 + the branching factor of eq. (6): one lane per
//                (frontier node, sample); Philox controls; Euler / RK4
//                integration of the whole segment (x'), with per-step validity
//                up to the first failing step (state box, then the swept box
//                against LDS-staged obstacles: a uniform grid for a double
//                integrator among many boxes, else candidate lists culled per
//                wave and per group of four lanes); sub-region map;
//                wave-aggregated n_valid / n_invalid atomics; acceptance; the
//                accepted samples staged per 64-lane wave tile.
//   k_post       the rest of the iteration in one launch: Alg. 3 (FreeVol,
//                Cov, Score and P_accept, eqs. 3-5, with an exact integer
//                score sum) in the region blocks; Alg. 4 (demote / promote)
//                fused with the compaction of the next frontier in the
//                node-set blocks, whose last chunk applies eq. (6); the
//                commit of V_U (ids in lane order) in the commit blocks.
// The step entry points run the same work as k_propagate + k_commit,
// k_region and k_nodesets.  Every kernel reads its sizes from device memory,
// so the host can enqueue several iterations without knowing them.
#include "kp_internal.h"

#include <hip/hip_ext.h>

#include "kp.h"
#include "kp_device.h"

namespace kp {

// ---------------------------------------------------------------------------
// wave / block helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long lanes_below() {
  return (1ull << __lane_id()) - 1ull;
}

// Wave reductions on the DPP path.  A DPP move is an operand modifier of a
// VALU instruction, so each step costs a few cycles instead of an LDS
// permute round trip; on a lone wave (small frontiers) these latencies add
// up to microseconds per tile.  The six steps: xor 1 and xor 2 inside each
// quad, the half-row and row mirrors (8- and 16-lane results), then the
// broadcasts of lane 15 into rows 1 and 3 and of lane 31 into rows 2 and 3.
// Lane 63 then holds the result of all 64 lanes, and the callers read it
// from there (wave-uniform).  Every lane of the wave must be active.
constexpr int kDppQuadXor1 = 0xb1;   // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4e;   // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;
constexpr int kDppBcast15 = 0x142;
constexpr int kDppBcast31 = 0x143;

// lanes of rows outside ROWS, and lanes without a source, get `old`
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_mov64(unsigned long long old,
                                                        unsigned long long v) {
  const uint32_t lo = dpp_mov<CTRL, ROWS>((uint32_t)old, (uint32_t)v);
  const uint32_t hi = dpp_mov<CTRL, ROWS>((uint32_t)(old >> 32), (uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

template <class Op>
__device__ __forceinline__ uint32_t dpp_reduce_u32(uint32_t v, uint32_t ident, Op op) {
  v = op(v, dpp_mov<kDppQuadXor1, 0xf>(ident, v));
  v = op(v, dpp_mov<kDppQuadXor2, 0xf>(ident, v));
  v = op(v, dpp_mov<kDppHalfMirror, 0xf>(ident, v));
  v = op(v, dpp_mov<kDppMirror, 0xf>(ident, v));
  v = op(v, dpp_mov<kDppBcast15, 0xa>(ident, v));
  v = op(v, dpp_mov<kDppBcast31, 0xc>(ident, v));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
template <class Op>
__device__ __forceinline__ unsigned long long dpp_reduce_u64(unsigned long long v,
                                                             unsigned long long ident, Op op) {
  v = op(v, dpp_mov64<kDppQuadXor1, 0xf>(ident, v));
  v = op(v, dpp_mov64<kDppQuadXor2, 0xf>(ident, v));
  v = op(v, dpp_mov64<kDppHalfMirror, 0xf>(ident, v));
  v = op(v, dpp_mov64<kDppMirror, 0xf>(ident, v));
  v = op(v, dpp_mov64<kDppBcast15, 0xa>(ident, v));
  v = op(v, dpp_mov64<kDppBcast31, 0xc>(ident, v));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  return dpp_reduce_u32(v, 0u, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
}
__device__ __forceinline__ float wave_min(float v) {
  return __uint_as_float(dpp_reduce_u32(__float_as_uint(v), 0x7f800000u, [](uint32_t a, uint32_t b) {
    return __float_as_uint(fminf(__uint_as_float(a), __uint_as_float(b)));
  }));
}
__device__ __forceinline__ float wave_max(float v) {
  return __uint_as_float(dpp_reduce_u32(__float_as_uint(v), 0xff800000u, [](uint32_t a, uint32_t b) {
    return __float_as_uint(fmaxf(__uint_as_float(a), __uint_as_float(b)));
  }));
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  return dpp_reduce_u64(v, 0ull, [](unsigned long long a, unsigned long long b) { return a + b; });
}
__device__ __forceinline__ unsigned long long wave_or_u64(unsigned long long v) {
  return dpp_reduce_u64(v, 0ull, [](unsigned long long a, unsigned long long b) { return a | b; });
}
__device__ __forceinline__ double wave_max_f64(double v) {
  return __longlong_as_double((long long)dpp_reduce_u64(
      (unsigned long long)__double_as_longlong(v), 0xfff0000000000000ull,
      [](unsigned long long a, unsigned long long b) {
        return (unsigned long long)__double_as_longlong(
            fmax(__longlong_as_double((long long)a), __longlong_as_double((long long)b)));
      }));
}

// min / max over the four lanes of each quad, in every lane of the quad
__device__ __forceinline__ float quad_min(float v) {
  v = fminf(v, __uint_as_float(dpp_mov<kDppQuadXor1, 0xf>(0x7f800000u, __float_as_uint(v))));
  return fminf(v, __uint_as_float(dpp_mov<kDppQuadXor2, 0xf>(0x7f800000u, __float_as_uint(v))));
}
__device__ __forceinline__ float quad_max(float v) {
  v = fmaxf(v, __uint_as_float(dpp_mov<kDppQuadXor1, 0xf>(0xff800000u, __float_as_uint(v))));
  return fmaxf(v, __uint_as_float(dpp_mov<kDppQuadXor2, 0xf>(0xff800000u, __float_as_uint(v))));
}

// Exclusive prefix of small per-lane counts (0..31) across the wave from five
// ballots of the count's bit planes.
__device__ __forceinline__ uint32_t wave_excl_small(uint32_t c, uint32_t* total) {
  const unsigned long long lo = lanes_below();
  uint32_t ex = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const unsigned long long m = __ballot((c >> b) & 1u);
    ex += (uint32_t)__popcll(m & lo) << b;
    tot += (uint32_t)__popcll(m) << b;
  }
  *total = tot;
  return ex;
}

// Decoupled look-back over per-tile status words: (30-bit epoch tag | 2-bit
// flag | 32-bit value); flag 1 = tile aggregate, 2 = inclusive prefix.  Run by
// one whole wave: lane l inspects tiles (t - 1 - l - 64 q), q < 4, so one
// probe round covers 256 predecessors; the nearest inclusive prefix ends the
// walk.  A tile only waits
// for tiles with smaller tickets, all held by running blocks, so the wait
// always ends; the spin bound only guards against a broken invariant.
__device__ uint32_t lookback_prefix_wave(unsigned long long* st, uint32_t tile, uint32_t agg,
                                         uint32_t epoch, uint32_t* err, uint32_t err_bit) {
  const unsigned long long tag = (unsigned long long)(epoch & 0x3fffffffu) << 34;
  const int lane = (int)__lane_id();
  if (tile == 0) {
    if (lane == 0)
      __hip_atomic_store(&st[0], tag | (2ull << 32) | agg, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    return 0u;
  }
  if (lane == 0)
    __hip_atomic_store(&st[tile], tag | (1ull << 32) | agg, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  // kLookWindows windows of 64 predecessors are requested per probe round, so
  // a walk past many unresolved tiles takes a quarter of the round trips;
  // the windows are then taken nearest first, and a window that is not yet
  // complete is requested again in the next round.
  constexpr int kLookWindows = 4;
  uint32_t excl = 0;
  int32_t base = (int32_t)tile - 1;
  uint32_t spins = 0;
  bool found = false;
  for (;;) {
    unsigned long long w[kLookWindows];
#pragma unroll
    for (int q = 0; q < kLookWindows; ++q) {
      const int32_t j = base - lane - 64 * q;
      w[q] = tag | (2ull << 32);  // before tile 0: an empty prefix
      if (j >= 0) w[q] = __hip_atomic_load(&st[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    bool stalled = false;
#pragma unroll
    for (int q = 0; q < kLookWindows; ++q) {
      if (found || stalled) continue;  // wave-uniform (from ballots)
      const uint32_t fl = (uint32_t)(w[q] >> 32) & 3u;
      const bool ready = ((uint32_t)(w[q] >> 34) == (epoch & 0x3fffffffu)) && fl != 0u;
      const unsigned long long pm = __ballot(ready && fl == 2u);
      const unsigned long long rm = __ballot(ready);
      const int limit = pm ? (__ffsll((long long)pm) - 1) : 63;
      const unsigned long long need = (limit == 63) ? ~0ull : ((1ull << (limit + 1)) - 1ull);
      if ((rm & need) != need) {
        stalled = true;
        continue;
      }
      excl += (uint32_t)wave_sum_u64(lane <= limit ? (unsigned long long)(uint32_t)w[q] : 0ull);
      if (pm) found = true;
      else base -= 64;
    }
    if (found) break;
    if (stalled) {
      if (++spins > (1u << 22)) {
        if (lane == 0) atomicOr(err, err_bit);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  if (lane == 0)
    __hip_atomic_store(&st[tile], tag | (2ull << 32) | (unsigned long long)(excl + agg),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

__device__ __forceinline__ uint32_t tile_total(unsigned long long* st, uint32_t ntiles) {
  if (ntiles == 0) return 0u;
  const unsigned long long w =
      __hip_atomic_load(&st[ntiles - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return (uint32_t)w;
}

// Block-wide exclusive offsets (kNodeBlock / 64 waves): per-wave totals in
// s_wt, then wave 0 resolves the tile's global prefix.  Returns the wave's offset inside the
// tile; *prefix receives the tile's global exclusive prefix.
__device__ __forceinline__ uint32_t block_offsets(uint32_t wave_total, uint32_t* s_wt,
                                                  uint32_t* s_pref, unsigned long long* st,
                                                  uint32_t tile, uint32_t epoch, uint32_t* err,
                                                  uint32_t* prefix, uint32_t err_bit,
                                                  uint32_t* tile_total = nullptr) {
  const int w = threadIdx.x >> 6;
  if (__lane_id() == 0) s_wt[w] = wave_total;
  __syncthreads();
  uint32_t off = 0, agg = 0;
#pragma unroll
  for (int k = 0; k < kNodeBlock / 64; ++k) {
    const uint32_t t = s_wt[k];
    off += (k < w) ? t : 0u;
    agg += t;
  }
  if (w == 0) {
    const uint32_t pre = lookback_prefix_wave(st, tile, agg, epoch, err, err_bit);
    if (__lane_id() == 0) *s_pref = pre;
  }
  __syncthreads();
  *prefix = *s_pref;
  if (tile_total) *tile_total = agg;
  return off;
}

// top 24 bits as a fraction in [0,1), then lo + (hi - lo) * r with one rounding
__device__ __forceinline__ float ctrl_map(uint32_t w, float lo, float hi) {
  const float r = (float)(w >> 8) * 0x1p-24f;
  return __builtin_fmaf(hi - lo, r, lo);
}

// ---------------------------------------------------------------------------
// dynamics (eq. 1) and one integration step (eq. 2), FP32
// ---------------------------------------------------------------------------
template <int DYN>
struct Dim;
template <>
struct Dim<KP_DYN_DI6> {
  static constexpr int n = 6, m = 3;
};
template <>
struct Dim<KP_DYN_QUAD12> {
  static constexpr int n = 12, m = 4;
};

// Per-step constants, copied out of Params once per kernel so that the step
// loop keeps them in registers instead of re-loading them from memory.
template <int DYN>
struct StepC {
  float h, inv_m, grav, inv_Ixx, inv_Iyy, inv_Izz, dIyz, dIzx, dIxy;
};

template <int DYN>
__device__ __forceinline__ StepC<DYN> load_step_consts(const Params& p) {
  StepC<DYN> s;
  s.h = p.h;
  s.inv_m = p.inv_m;
  s.grav = p.grav;
  s.inv_Ixx = p.inv_Ixx;
  s.inv_Iyy = p.inv_Iyy;
  s.inv_Izz = p.inv_Izz;
  s.dIyz = p.dIyz;
  s.dIzx = p.dIzx;
  s.dIxy = p.dIxy;
  return s;
}

template <class PP>
__device__ __forceinline__ void deriv_di(const PP&, const float* x, const float* u, float* dx) {
  dx[0] = x[3];
  dx[1] = x[4];
  dx[2] = x[5];
  dx[3] = u[0];
  dx[4] = u[1];
  dx[5] = u[2];
}

// sin and cos without branches for |x| up to ~1e4 (the state box bounds the
// angles far below that): x = k * pi/2 + r, |r| <= pi/4, with pi/2 split into
// three FP32 parts (Cody-Waite reduction, each product folded into one fused
// multiply-add); then the Taylor polynomials of sin (to degree 9) and cos (to
// degree 10) on [-pi/4, pi/4], whose truncation errors are below 2e-9 and
// 1.2e-10; the quadrant k mod 4 swaps and negates.  Coefficients are 1/n!
// rounded to FP32.  Measured against FP64 sin/cos on [-1000, 1000]: at most
// 1.5 ulp, absolute error below 8e-8.
__device__ __forceinline__ void sincos_rr(float x, float* s, float* c) {
  const float k = rintf(x * 0x1.45f306p-1f);  // 2/pi
  float r = __builtin_fmaf(-k, 0x1.921fb6p+0f, x);
  r = __builtin_fmaf(-k, -0x1.777a5cp-25f, r);
  r = __builtin_fmaf(-k, -0x1.ee59dap-50f, r);
  const float r2 = r * r;
  float ps = __builtin_fmaf(r2, 0x1.71de3ap-19f, -0x1.a01a02p-13f);
  ps = __builtin_fmaf(r2, ps, 0x1.111112p-7f);
  ps = __builtin_fmaf(r2, ps, -0x1.555556p-3f);
  const float sr = __builtin_fmaf(r * r2, ps, r);
  float pc = __builtin_fmaf(r2, -0x1.27e4fcp-22f, 0x1.a01a02p-16f);
  pc = __builtin_fmaf(r2, pc, -0x1.6c16c2p-10f);
  pc = __builtin_fmaf(r2, pc, 0x1.555556p-5f);
  pc = __builtin_fmaf(r2, pc, -0.5f);
  const float cr = __builtin_fmaf(r2, pc, 1.0f);
  const int q = (int)k;
  const float sv = (q & 1) ? cr : sr;
  const float cv = (q & 1) ? sr : cr;
  *s = __uint_as_float(__float_as_uint(sv) ^ (((uint32_t)q & 2u) << 30));
  *c = __uint_as_float(__float_as_uint(cv) ^ (((uint32_t)(q + 1) & 2u) << 30));
}

// sin and cos of a tilt angle (roll, pitch) or of an RK4 stage's yaw
// increment.  For |x| <= 1.8, near-minimax polynomials on [-1.8, 1.8] of
// degree 9 (sin, odd) and 10 (cos, even) apply with no reduction: measured
// in FP32 Horner form against FP64 sin / cos on 2e6 points, sin is within
// 2.6 ulp and cos within 1.1e-7 absolute.  A state inside the valid box keeps
// every stage's angles in that range, but a segment that has left the box
// is still integrated to its end (x' of Alg. 2), and its angles can grow
// without bound; a wave with any larger angle also runs the full reduction
// for those lanes.
__device__ __forceinline__ void sincos_tilt(float x, float* s, float* c) {
  const float t = x * x;
  float ps = __builtin_fmaf(t, 0x1.5880bep-19f, -0x1.9f1b8cp-13f);
  ps = __builtin_fmaf(t, ps, 0x1.110dcep-7f);
  ps = __builtin_fmaf(t, ps, -0x1.555554p-3f);
  float sv = __builtin_fmaf(x * t, ps, x);
  float pc = __builtin_fmaf(t, -0x1.13d974p-22f, 0x1.9f1102p-16f);
  pc = __builtin_fmaf(t, pc, -0x1.6c10e4p-10f);
  pc = __builtin_fmaf(t, pc, 0x1.55553ep-5f);
  pc = __builtin_fmaf(t, pc, -0.5f);
  float cv = __builtin_fmaf(t, pc, 1.0f);
  const bool big = !(__builtin_fabsf(x) <= 1.8f);  // NaN too
  if (__builtin_expect(__ballot(big) != 0ull, 0)) {
    float s2, c2;
    sincos_rr(x, &s2, &c2);
    sv = big ? s2 : sv;
    cv = big ? c2 : cv;
  }
  *s = sv;
  *c = cv;
}

// rigid-body quadcopter, ZYX Euler angles, inertial velocity, body rates
template <class PP>
__device__ __forceinline__ void deriv_quad(const PP& p, const float* x, const float* u,
                                           float* dx) {
  float sf, cf, st, ct, sp, cp;
  sincos_tilt(x[3], &sf, &cf);
  sincos_tilt(x[4], &st, &ct);
  sincos_rr(x[5], &sp, &cp);
  const float ict = __builtin_amdgcn_rcpf(ct);  // 1 ulp; |theta| stays far from pi/2
  const float P = x[9], Q = x[10], R = x[11];
  const float a = __builtin_fmaf(Q, sf, R * cf);
  dx[0] = x[6];
  dx[1] = x[7];
  dx[2] = x[8];
  dx[3] = __builtin_fmaf(a * st, ict, P);
  dx[4] = __builtin_fmaf(Q, cf, -(R * sf));
  dx[5] = a * ict;
  const float tm = u[0] * p.inv_m;
  const float cfst = cf * st;
  dx[6] = tm * __builtin_fmaf(cfst, cp, sf * sp);
  dx[7] = tm * __builtin_fmaf(cfst, sp, -(sf * cp));
  dx[8] = __builtin_fmaf(tm, cf * ct, -p.grav);
  dx[9] = __builtin_fmaf(p.dIyz * Q, R, u[1]) * p.inv_Ixx;
  dx[10] = __builtin_fmaf(p.dIzx * P, R, u[2]) * p.inv_Iyy;
  dx[11] = __builtin_fmaf(p.dIxy * P, Q, u[3]) * p.inv_Izz;
}

// the quadcopter derivative with sin / cos of the yaw angle supplied
template <class PP>
__device__ __forceinline__ void deriv_quad_y(const PP& p, const float* x, const float* u, float sp,
                                             float cp, float* dx) {
  float sf, cf, st, ct;
  sincos_tilt(x[3], &sf, &cf);
  sincos_tilt(x[4], &st, &ct);
  const float ict = __builtin_amdgcn_rcpf(ct);
  const float P = x[9], Q = x[10], R = x[11];
  const float a = __builtin_fmaf(Q, sf, R * cf);
  dx[0] = x[6];
  dx[1] = x[7];
  dx[2] = x[8];
  dx[3] = __builtin_fmaf(a * st, ict, P);
  dx[4] = __builtin_fmaf(Q, cf, -(R * sf));
  dx[5] = a * ict;
  const float tm = u[0] * p.inv_m;
  const float cfst = cf * st;
  dx[6] = tm * __builtin_fmaf(cfst, cp, sf * sp);
  dx[7] = tm * __builtin_fmaf(cfst, sp, -(sf * cp));
  dx[8] = __builtin_fmaf(tm, cf * ct, -p.grav);
  dx[9] = __builtin_fmaf(p.dIyz * Q, R, u[1]) * p.inv_Ixx;
  dx[10] = __builtin_fmaf(p.dIzx * P, R, u[2]) * p.inv_Iyy;
  dx[11] = __builtin_fmaf(p.dIxy * P, Q, u[3]) * p.inv_Izz;
}

// sin / cos of psi0 + d from those of psi0 (angle addition); d is an RK4
// stage's yaw increment, so sin d and cos d take the short polynomials
__device__ __forceinline__ void sincos_shift(float s0, float c0, float d, float* s, float* c) {
  float sd, cd;
  sincos_tilt(d, &sd, &cd);
  *s = __builtin_fmaf(s0, cd, c0 * sd);
  *c = __builtin_fmaf(c0, cd, -(s0 * sd));
}

template <int DYN, class PP>
__device__ __forceinline__ void deriv(const PP& p, const float* x, const float* u, float* dx) {
  if constexpr (DYN == KP_DYN_DI6) deriv_di(p, x, u, dx);
  else deriv_quad(p, x, u, dx);
}

// Yaw frame of a quadcopter segment.  The yaw is unbounded (the state box
// allows hundreds of radians), and an FP32 angle near 16 rad is stored to
// about 1e-6 rad, an error that the thrust direction turns into velocity
// errors of ~1e-5 over a segment when it accumulates step by step.  So a
// segment keeps its start angle psi0 (its parent's stored value, an exact
// input) with that angle's sine and cosine, and integrates the offset
// d = psi - psi0, which stays small; sin / cos of psi0 + d follow by angle
// addition, and the state's yaw is psi0 + d rounded once.
struct YawFrame {
  float s0, c0, psi0, d;
};

template <int DYN, int INTEG, class PP>
__device__ __forceinline__ void integ_step(const PP& p, float* x, const float* u, YawFrame& y) {
  constexpr int n = Dim<DYN>::n;
  const float h = p.h;
  if constexpr (DYN == KP_DYN_QUAD12 && INTEG == KP_INT_EULER) {
    float sp, cp, k1[n];
    sincos_shift(y.s0, y.c0, y.d, &sp, &cp);
    deriv_quad_y(p, x, u, sp, cp, k1);
#pragma unroll
    for (int i = 0; i < n; ++i)
      if (i != 5) x[i] = __builtin_fmaf(h, k1[i], x[i]);
    y.d = __builtin_fmaf(h, k1[5], y.d);
    x[5] = y.psi0 + y.d;
  } else if constexpr (INTEG == KP_INT_EULER) {
    float k1[n];
    deriv<DYN>(p, x, u, k1);
#pragma unroll
    for (int i = 0; i < n; ++i) x[i] = __builtin_fmaf(h, k1[i], x[i]);
  } else if constexpr (DYN == KP_DYN_QUAD12) {
    // the step's yaw from the segment frame; the stages shift it by their
    // increments
    const float hh = 0.5f * h;
    const float h6 = h * (1.0f / 6.0f);
    float sp0, cp0, sp, cp;
    sincos_shift(y.s0, y.c0, y.d, &sp0, &cp0);
    float t[n], k[n], acc[n];
    deriv_quad_y(p, x, u, sp0, cp0, k);
#pragma unroll
    for (int i = 0; i < n; ++i) {
      acc[i] = k[i];
      t[i] = __builtin_fmaf(hh, k[i], x[i]);
    }
    sincos_shift(sp0, cp0, hh * k[5], &sp, &cp);
    deriv_quad_y(p, t, u, sp, cp, k);
#pragma unroll
    for (int i = 0; i < n; ++i) {
      acc[i] = __builtin_fmaf(2.0f, k[i], acc[i]);
      t[i] = __builtin_fmaf(hh, k[i], x[i]);
    }
    sincos_shift(sp0, cp0, hh * k[5], &sp, &cp);
    deriv_quad_y(p, t, u, sp, cp, k);
#pragma unroll
    for (int i = 0; i < n; ++i) {
      acc[i] = __builtin_fmaf(2.0f, k[i], acc[i]);
      t[i] = __builtin_fmaf(h, k[i], x[i]);
    }
    sincos_shift(sp0, cp0, h * k[5], &sp, &cp);
    deriv_quad_y(p, t, u, sp, cp, k);
#pragma unroll
    for (int i = 0; i < n; ++i)
      if (i != 5) x[i] = __builtin_fmaf(h6, acc[i] + k[i], x[i]);
    y.d = __builtin_fmaf(h6, acc[5] + k[5], y.d);
    x[5] = y.psi0 + y.d;
  } else {
    const float hh = 0.5f * h;
    const float h6 = h * (1.0f / 6.0f);
    float k1[n];
    deriv<DYN>(p, x, u, k1);
    float t[n], k[n], acc[n];
#pragma unroll
    for (int i = 0; i < n; ++i) {
      acc[i] = k1[i];
      t[i] = __builtin_fmaf(hh, k1[i], x[i]);
    }
    deriv<DYN>(p, t, u, k);
#pragma unroll
    for (int i = 0; i < n; ++i) {
      acc[i] = __builtin_fmaf(2.0f, k[i], acc[i]);
      t[i] = __builtin_fmaf(hh, k[i], x[i]);
    }
    deriv<DYN>(p, t, u, k);
#pragma unroll
    for (int i = 0; i < n; ++i) {
      acc[i] = __builtin_fmaf(2.0f, k[i], acc[i]);
      t[i] = __builtin_fmaf(h, k[i], x[i]);
    }
    deriv<DYN>(p, t, u, k);
#pragma unroll
    for (int i = 0; i < n; ++i) x[i] = __builtin_fmaf(h6, acc[i] + k[i], x[i]);
  }
}

template <int DYN, class PP>
__device__ __forceinline__ bool state_ok(const PP& p, const float* x) {
  constexpr int n = Dim<DYN>::n;
  float lo[n], hi[n];
#pragma unroll
  for (int i = 0; i < n; ++i) {
    lo[i] = p.x_lo[i];
    hi[i] = p.x_hi[i];
  }
  bool ok = true;
#pragma unroll
  for (int i = 0; i < n; ++i) ok = ok && (x[i] >= lo[i]) && (x[i] <= hi[i]);
  return ok;  // NaN fails both comparisons
}

// the same test with the box read from LDS (lo at b[0..11], hi at b[12..23]):
// six 16-byte broadcast reads issued together instead of dependent scalar loads
template <int DYN>
__device__ __forceinline__ bool state_ok_lds(const float* __restrict__ b, const float* x) {
  constexpr int n = Dim<DYN>::n;
  float bb[24];
  const float4* b4 = reinterpret_cast<const float4*>(b);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float4 v = b4[i];
    bb[4 * i] = v.x;
    bb[4 * i + 1] = v.y;
    bb[4 * i + 2] = v.z;
    bb[4 * i + 3] = v.w;
  }
  bool ok = true;
#pragma unroll
  for (int i = 0; i < n; ++i) ok &= (x[i] >= bb[i]) & (x[i] <= bb[12 + i]);
  return ok;
}

// The quadcopter test when the box is symmetric about zero in every
// coordinate but position (lo = -hi, checked on the host): lo <= x <= hi is
// then exactly |x| <= hi (negation is exact, and a NaN fails), one compare
// with a free absolute-value modifier instead of two; position keeps both.
__device__ __forceinline__ bool state_ok_lds_sym(const float* __restrict__ b, const float* x) {
  const float4* b4 = reinterpret_cast<const float4*>(b);
  const float4 lo = b4[0], h0 = b4[3], h1 = b4[4], h2 = b4[5];
  const float hi[12] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w, h2.x, h2.y, h2.z, h2.w};
  bool ok = (x[0] >= lo.x) & (x[1] >= lo.y) & (x[2] >= lo.z);
#pragma unroll
  for (int i = 0; i < 3; ++i) ok &= x[i] <= hi[i];
#pragma unroll
  for (int i = 3; i < 12; ++i) ok &= __builtin_fabsf(x[i]) <= hi[i];
  return ok;
}

// fine cell (region * 64 + sub-cell) of a finite position, clamped to W
__device__ __forceinline__ uint32_t cell_of(const Params& p, float px, float py, float pz) {
  const float q[3] = {px, py, pz};
  int c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float t = (q[a] - p.w_lo[a]) * p.inv_w[a];
    t = fminf(fmaxf(t, 0.0f), (float)(p.na[a] - 1));
    c[a] = (int)floorf(t);
  }
  const int S = p.S;
  const uint32_t region = (uint32_t)(((c[2] / S) * p.G[1] + (c[1] / S)) * p.G[0] + (c[0] / S));
  const uint32_t local = (uint32_t)(((c[2] % S) * S + (c[1] % S)) * S + (c[0] % S));
  return region * 64u + local;
}

// ---------------------------------------------------------------------------
// k_zero / k_root / k_set_ctl: (re)initialisation, Alg. 1's set-up of the
// tree, V_E and P_accept
// ---------------------------------------------------------------------------
__global__ void k_zero(const Env* __restrict__ env) {
  const Params& p = env->p;
  const Dev& d = env->d;
  const int stride = gridDim.x * blockDim.x;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < p.R; r += stride) {
    d.nv[r] = 0ull;
    d.ni[r] = 0ull;
    d.visited[r] = 0ull;
    d.thr[r] = 1ull << 32;
    d.avail[r] = 0;
  }
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < d.tiles_node; t += stride) {
    d.st_front[t] = 0ull;
    d.st_nodes[t] = 0ull;
  }
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < 2 * d.nchunk; t += stride) d.ssum[t] = 0u;
}

__device__ void clear_counters(Ctl* c) {
  c->tk_front = c->tk_nodes = 0u;
  c->bd_front = c->bd_nodes = 0u;
  c->err = 0u;
  c->f_expl = c->f_base = 0;
  c->goal_hit = 0u;
  for (int g = 0; g < kGroups; ++g) {
    c->tot[g].lanes = c->tot[g].valid = c->tot[g].steps = c->tot[g].box = 0ull;
    c->tot[g].checked = 0ull;
    c->tkp[g].v = 0u;
  }
}

__global__ void k_root(const Env* __restrict__ env, Vec12 xi) {
  const Params& p = env->p;
  const Dev& d = env->d;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  Ctl* c = d.ctl;
  for (int k = 0; k < p.n; ++k) d.x[(size_t)k * d.capP] = xi.v[k];
  for (int k = 0; k < p.m; ++k) d.u[(size_t)k * d.capP] = 0.0f;
  const uint32_t cl = cell_of(p, xi.v[0], xi.v[1], xi.v[2]);
  d.parent[0] = -1;
  d.cell[0] = cl;
  d.flag[0] = 1;
  d.birth[0] = -1;
  d.sample[0] = 0;
  d.visited[cl >> 6] = 1ull << (cl & 63u);
  d.avail[cl >> 6] = 1;
  const float dx = xi.v[0] - p.goal_c[0], dy = xi.v[1] - p.goal_c[1], dz = xi.v[2] - p.goal_c[2];
  const bool in_goal = dx * dx + dy * dy + dz * dz <= p.goal_r2;
  c->N = 1;
  c->nF = 0;
  c->lambda = 0;
  c->lanes = 0;
  c->nU = 0;
  c->it = 0;
  c->goal_id = in_goal ? 0 : kNoGoal;
  c->done = in_goal ? KP_SOLVED : 0;
  c->epoch = c->epoch + 1u;
  c->iters_done = 0u;
  clear_counters(c);
}

// state loaded from the host: counters for |T| = N at iteration `it`
__global__ void k_set_ctl(const Env* __restrict__ env, int32_t N, int32_t it) {
  const Dev& d = env->d;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  Ctl* c = d.ctl;
  c->N = N;
  c->nF = 0;
  c->lambda = 0;
  c->lanes = 0;
  c->nU = 0;
  c->it = it;
  c->goal_id = kNoGoal;
  c->done = 0;
  c->epoch = c->epoch + 1u;
  clear_counters(c);
  for (int j = 0; j < 2 * d.nchunk; ++j) d.ssum[j] = 0u;
}

// flag bytes of the kNodesPerThread nodes a thread holds, as 32-bit words
constexpr int kFlagWords = kNodesPerThread / 4;
static_assert(kNodesPerThread == 4 || kNodesPerThread == 16, "flag word loads");
__device__ __forceinline__ void load_flag_words(const uint8_t* f, uint32_t* w) {
  if constexpr (kNodesPerThread == 16) {
    const uint4 v = *reinterpret_cast<const uint4*>(f);
    w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
  } else {
    w[0] = *reinterpret_cast<const uint32_t*>(f);
  }
}
__device__ __forceinline__ void store_flag_words(uint8_t* f, const uint32_t* w) {
  if constexpr (kNodesPerThread == 16) {
    *reinterpret_cast<uint4*>(f) = make_uint4(w[0], w[1], w[2], w[3]);
  } else {
    *reinterpret_cast<uint32_t*>(f) = w[0];
  }
}

// ---------------------------------------------------------------------------
// frontier compaction shared by k_frontier and k_nodesets
// ---------------------------------------------------------------------------
// E-bits of the nodes held by this thread -> F, in ascending id order.
// Returns the number of E nodes up to and including this tile.
__device__ __forceinline__ uint32_t compact_frontier(const Dev& d, unsigned long long* st,
                                                     uint32_t ebits, uint32_t base, uint32_t tile,
                                                     uint32_t epoch, uint32_t* s_wt,
                                                     uint32_t* s_pref) {
  uint32_t wt, agg;
  const uint32_t c = __popc(ebits);
  const uint32_t ex = wave_excl_small(c, &wt);
  uint32_t prefix;
  const uint32_t woff =
      block_offsets(wt, s_wt, s_pref, st, tile, epoch, &d.ctl->err, &prefix,
                    st == d.st_nodes ? 4u : 1u, &agg);
  uint32_t pos = prefix + woff + ex;
  while (ebits) {
    const int k = __ffs(ebits) - 1;
    d.F[pos++] = (int32_t)(base + k);
    ebits &= ebits - 1u;
  }
  return prefix + agg;
}

// last-block finalisation of the frontier: |V_E|, eq. (6), termination codes
__device__ __forceinline__ void finalize_frontier(const Params& p, Ctl* c, uint32_t nF,
                                                  int32_t N) {
  int32_t lam = 0;
  if (nF > 0) {
    lam = (p.cap - N) / (int32_t)nF;
    if (lam > p.lambda_max) lam = p.lambda_max;
  }
  c->nF = (int32_t)nF;
  c->f_expl = (int32_t)nF;
  c->f_base = 0;
  c->lambda = lam;
  c->lanes = (int32_t)nF * lam;
  if (c->done == 0) {
    if (nF == 0) c->done = KP_FRONTIER_EMPTY;
    else if (lam == 0) c->done = KP_TREE_FULL;
  }
}

__global__ __launch_bounds__(kNodeBlock) void k_frontier(const Env* __restrict__ env) {
  const Params& p = env->p;
  const Dev& d = env->d;
  Ctl* c = d.ctl;
  const int32_t N = c->N;
  const int done = c->done;
  const uint32_t epoch = c->epoch;
  const uint32_t ntiles = done ? 0u : (uint32_t)((N + kNodeTile - 1) / kNodeTile);
  __shared__ uint32_t s_tile, s_pref, s_wt[kNodeBlock / 64];
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(&c->tk_front, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) break;
    const uint32_t base = tile * kNodeTile + threadIdx.x * kNodesPerThread;
    uint32_t fw[kFlagWords];
    load_flag_words(d.flag + base, fw);
    uint32_t eb = 0;
#pragma unroll
    for (int k = 0; k < kNodesPerThread; ++k)
      if (base + k < (uint32_t)N && ((fw[k >> 2] >> (8 * (k & 3))) & 0xffu)) eb |= 1u << k;
    compact_frontier(d, d.st_front, eb, base, tile, epoch, s_wt, &s_pref);
    __syncthreads();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t prev = atomicAdd(&c->bd_front, 1u);
    if (prev == gridDim.x - 1u) {
      __threadfence();
      if (!done) finalize_frontier(p, c, tile_total(d.st_front, ntiles), N);
      c->tk_front = 0u;
      c->bd_front = 0u;
    }
  }
}

// ---------------------------------------------------------------------------
// k_propagate: Alg. 2
// ---------------------------------------------------------------------------
// LDS of a propagate block: the obstacle table ((n_obs + 1) boxes of six
// floats; box n_obs is a sentinel that no segment touches), then per wave a
// union candidate list, kGroupsPerWave group lists and their counts.
constexpr int kLaneGroup = 4;                       // lanes per culling group
constexpr int kGroupsPerWave = 64 / kLaneGroup;
constexpr int kGroupCap = 30;                       // candidates a group list holds
constexpr int kGroupStride = kGroupCap + 2;         // + room to pad to an even length
constexpr uint32_t kGroupCull = 8;                  // longer union lists are split per group
__host__ __device__ constexpr int union_stride(int n_obs) { return (n_obs + 2 + 3) & ~3; }
__host__ __device__ constexpr size_t wave_lds_bytes(int n_obs) {
  return (size_t)union_stride(n_obs) * 2 + (size_t)kGroupsPerWave * kGroupStride * 2 +
         (size_t)kGroupsPerWave * 4;
}
constexpr int kBoundsFloats = 2 * 12;   // state box (lo[12], hi[12]) at the start of the block LDS
// LDS of a propagate block.  Quadcopter: state box, obstacle table, per-wave
// candidate lists.  Double integrator: state box, obstacle table, and the
// obstacle grid (grid_words u16 words: cell offsets, then obstacle ids).
constexpr size_t prop_lds_bytes(int dyn, int n_obs, int grid_words, int waves = 0) {
  return kBoundsFloats * sizeof(float) + (size_t)(n_obs + 1) * 6 * sizeof(float) +
         (grid_words > 0
              ? (size_t)((grid_words + 1) & ~1) * 2
              : (size_t)(waves > 0 ? waves : prop_block(dyn) / 64) * wave_lds_bytes(n_obs));
}
// gfx950 gives a workgroup up to 160 KiB of LDS
static_assert(prop_lds_bytes(KP_DYN_QUAD12, KP_MAX_OBSTACLES, 0) <= 150 * 1024 &&
                  prop_lds_bytes(KP_DYN_DI6, KP_MAX_OBSTACLES, kGridMaxWords) <= 150 * 1024 &&
                  prop_lds_bytes(KP_DYN_DI6, kGridMinObstacles, 0) <= 150 * 1024,
              "propagate LDS (with the static arrays) above 160 KiB");
size_t propagate_lds_bytes(int dyn, int n_obs, int grid_words) {
  return prop_lds_bytes(dyn, n_obs, grid_words);
}
size_t queue_lds_bytes(int dyn, int n_obs, int grid_words) {
  return prop_lds_bytes(dyn, n_obs, grid_words, kQueueBlock / 64);
}
static_assert(prop_lds_bytes(KP_DYN_QUAD12, KP_MAX_OBSTACLES, 0, kQueueBlock / 64) <= 150 * 1024,
              "queue kernel LDS (with the static arrays of the post body) above 160 KiB");


// Separation of two closed boxes: the largest gap along any axis between a
// face of one and the facing face of the other.  The boxes intersect
// (touching included) iff the separation is <= 0; for finite operands
// a - b <= 0 holds exactly when a <= b, so this is the same test as six
// comparisons, computed without lane masks.
__device__ __forceinline__ float box_separation(float lx, float ly, float lz, float hx, float hy,
                                                float hz, const float2* ob) {
  const float2 a = ob[0], b = ob[1], c = ob[2];  // (lo x, lo y), (lo z, hi x), (hi y, hi z)
  const float s0 = fmaxf(fmaxf(lx - b.y, a.x - hx), ly - c.x);
  const float s1 = fmaxf(fmaxf(a.y - hy, lz - c.y), b.x - hz);
  return fmaxf(s0, s1);
}

// Box of every position a double-integrator segment passes through.  With
// constant control the positions are a quadratic in the step index j:
// explicit Euler gives p_j = p_0 + j h v_0 + h^2 u j (j - 1) / 2, and RK4,
// exact on this system, p_0 + j h v_0 + (j h)^2 u / 2.  Per axis the range
// over j in [0, K] is spanned by the two ends and, when it lies inside, the
// vertex.  The box is widened by a bound on the rounding of K FP32 steps
// (each at most a few units in the last place of coordinates below M), so
// it holds the positions the kernel computes, not only the exact ones.
template <int INTEG>
__device__ __forceinline__ void segment_box_di(const float* x, const float* u, int K, float h,
                                               float* lo, float* hi) {
  const float kf = (float)K;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float A = 0.5f * h * h * u[a];
    const float B = (INTEG == KP_INT_EULER) ? __builtin_fmaf(h, x[3 + a], -A) : h * x[3 + a];
    const float C = x[a];
    const float fk = __builtin_fmaf(kf, __builtin_fmaf(kf, A, B), C);
    float l = fminf(C, fk), g = fmaxf(C, fk);
    // vertex at j* = -B / (2A), value C - B^2 / (4A)
    const float js = -B / (2.0f * A);
    const bool inside = A != 0.0f && js > 0.0f && js < kf;
    const float fv = C - (B * B) / (4.0f * A);
    l = inside ? fminf(l, fv) : l;
    g = inside ? fmaxf(g, fv) : g;
    const float eps = 1e-3f + (kf + 4.0f) * 1e-6f * (1.0f + fmaxf(fabsf(l), fabsf(g)));
    lo[a] = l - eps;
    hi[a] = g + eps;
  }
}

// Cell index floor(t) of a grid coordinate t, clamped to [0, ncell - 1]
// (t is finite: the swept boxes tested lie inside the state box).
__device__ __forceinline__ int clamp_cell(float t, int ncell) {
  const int c = (int)floorf(t);
  return c < 0 ? 0 : (c > ncell - 1 ? ncell - 1 : c);
}

// One propagate launch's work for block vb of a grid of vg blocks of PB
// threads (a kernel's own blockIdx.x and gridDim.x, or block 0 of 1 when one
// workgroup runs a whole query).
template <int DYN, int INTEG, bool SYM, int PB>
__device__ __forceinline__ void propagate_body(const Env* __restrict__ env, TraceRec* trace,
                                               uint32_t vb, uint32_t vg) {
  const Params& p = env->p;
  const Dev& d = env->d;
  constexpr int n = Dim<DYN>::n;
  constexpr int m = Dim<DYN>::m;
  constexpr int kWaves = PB / 64;
  extern __shared__ float lds[];
  Ctl* c = d.ctl;
  const int done = c->done;
  const int32_t lanes = c->lanes;
  const int32_t lam = c->lambda;
  const uint32_t it = (uint32_t)c->it;
  const int32_t f_expl = c->f_expl, f_base = c->f_base;
  // the node-set ticket counter, last used by the previous iteration's node
  // pass, starts from zero for the next one; the iteration's sizes are
  // copied for k_post
  if (vb == 0 && threadIdx.x == 0) {
    c->tk_nodes = 0u;
    c->rg_max = 0ull;
    c->rg_sum = 0ull;
    c->rg_cnt_max = c->rg_cnt_sum = c->rg_cnt_thr = 0u;
    c->sN = c->N;
    c->sit = (int32_t)it;
    c->sdone = done;
    c->sepoch = c->epoch;
    c->slanes = lanes;
    c->slam = lam;
  }
  uint32_t* ssum_it = d.ssum + (size_t)(it & 1u) * (size_t)d.nchunk;
  // tiles are single waves: each wave takes 64 lanes at a time from the ticket
  const uint32_t ntiles = done ? 0u : (uint32_t)((lanes + 63) / 64);
  const StepC<DYN> sc = load_step_consts<DYN>(p);
  const int K = p.K;
  const float margin = p.margin;
  const int n_obs = p.n_obs;
  const int wave = threadIdx.x >> 6;
  // a double integrator among more than kGridMinObstacles boxes finds its
  // obstacles through the grid at each step; otherwise (and always for the
  // quadcopter) a wave culls them once per tile into candidate lists
  const bool use_grid = DYN == KP_DYN_DI6 && p.og_n[0] > 0;
  // obstacle k in LDS: lo x, lo y, lo z, hi x, hi y, hi z (6 floats, read as 3 float2)
  float* bnd = lds;  // state box
  float* otab = lds + kBoundsFloats;
  const float2* obox = reinterpret_cast<const float2*>(otab);
  char* after_tab = reinterpret_cast<char*>(otab) + (size_t)(n_obs + 1) * 6 * sizeof(float);
  // double integrator: the obstacle grid (cell offsets, then obstacle ids)
  uint16_t* goff = reinterpret_cast<uint16_t*>(after_tab);
  const int gnx = p.og_n[0], gny = p.og_n[1];
  const uint16_t* gent = goff + gnx * gny * p.og_n[2] + 1;
  // quadcopter: this wave's candidate lists
  char* wlds = after_tab + (size_t)wave * wave_lds_bytes(n_obs);
  uint16_t* cand = reinterpret_cast<uint16_t*>(wlds);
  uint16_t* glist = cand + union_stride(n_obs);
  uint32_t* gcnt = reinterpret_cast<uint32_t*>(glist + kGroupsPerWave * kGroupStride);
  // per-wave running totals (wave-uniform), flushed once per block
  unsigned long long t_lanes = 0, t_valid = 0, t_steps = 0, t_box = 0, t_checked = 0;

  // A wave's first tile is wave * vg + slot(block): the first vg tiles go to
  // wave 0 of every block, the next ones to wave 1, and so on, so that a
  // launch with fewer tiles than the grid has waves runs one wave per block,
  // spread over the compute units.  Workgroups are dispatched to the 8 XCDs
  // round robin (block b on XCD b mod 8), and neighbouring tiles read
  // neighbouring parents, whose 128-byte lines they share: slot(b) gives
  // XCD x the contiguous slots x * vg/8 .. (x+1) * vg/8 - 1, so neighbours
  // meet in one L2 (the host makes vg a multiple of 8, or below 8).  Later
  // tiles come from per-group ticket counters: group q (block index mod ng)
  // hands out tiles nwaves + ng * k + q.  No burst of tickets at launch, and
  // each counter sees about 1/ng of the requests.  A block whose first tiles
  // are all past the end has nothing to do (an oversized grid costs no
  // atomics).
  const uint32_t nwaves = vg * kWaves;
  const uint32_t ng = vg < (uint32_t)kGroups ? vg : (uint32_t)kGroups;
  const uint32_t grp = vb % ng;
  const uint32_t slot = (vg % 8u == 0u) ? (vb % 8u) * (vg / 8u) + vb / 8u : vb;
  if (slot >= ntiles) return;
  // the obstacle table: coalesced reads of the six component arrays, each
  // value stored at its box's slot
  // (both copies issue eight loads per thread before their LDS stores, so
  // the loads' round trips overlap instead of following one another)
  constexpr int kStage = 8;
  for (int k0 = threadIdx.x; k0 < 6 * n_obs; k0 += kStage * PB) {
    float v[kStage];
#pragma unroll
    for (int j = 0; j < kStage; ++j) {
      const int k = k0 + j * PB;
      v[j] = (k < 6 * n_obs) ? d.obs[k] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kStage; ++j) {
      const int k = k0 + j * PB;
      const int comp = (k >= n_obs) + (k >= 2 * n_obs) + (k >= 3 * n_obs) + (k >= 4 * n_obs) +
                       (k >= 5 * n_obs);
      if (k < 6 * n_obs) otab[6 * (k - comp * n_obs) + comp] = v[j];
    }
  }
  if (use_grid) {
    // the grid's u16 words, copied two at a time (the device copy is padded
    // to an even count)
    const int nw2 = (p.og_words + 1) >> 1;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(d.og);
    uint32_t* dst = reinterpret_cast<uint32_t*>(goff);
    for (int k0 = threadIdx.x; k0 < nw2; k0 += kStage * PB) {
      uint32_t v[kStage];
#pragma unroll
      for (int j = 0; j < kStage; ++j) {
        const int k = k0 + j * PB;
        v[j] = (k < nw2) ? src[k] : 0u;
      }
#pragma unroll
      for (int j = 0; j < kStage; ++j) {
        const int k = k0 + j * PB;
        if (k < nw2) dst[k] = v[j];
      }
    }
  }
  if (threadIdx.x < 6) otab[6 * n_obs + threadIdx.x] = (threadIdx.x < 3) ? 3.0e38f : -3.0e38f;
  if (threadIdx.x < (unsigned)n) {
    bnd[threadIdx.x] = p.x_lo[threadIdx.x];
    bnd[12 + threadIdx.x] = p.x_hi[threadIdx.x];
  }
  __syncthreads();

  uint32_t next = (uint32_t)wave * vg + slot;
  for (;;) {
    const uint32_t tile = next;
    if (tile >= ntiles) break;

    const int32_t g = (int32_t)(tile * 64u + __lane_id());
    const bool active = g < lanes;
    int32_t e = 0, s = 0, f = 0;
    float x[n];
    float u[m];
    uint32_t w_acc = 0;
    int kl = K;  // this segment's steps
    if (active) {
      e = g / lam;
      s = g - e * lam;
      f = frontier_node(d.F, e, f_expl, f_base);
#pragma unroll
      for (int k = 0; k < n; ++k) x[k] = d.x[(size_t)k * d.capP + f];
      const U4 w = philox(it, (uint32_t)f, (uint32_t)s, 0u, p.key0, p.key1);
#pragma unroll
      for (int j = 0; j < m; ++j) u[j] = ctrl_map(w.w[j], p.u_lo[j], p.u_hi[j]);
      if constexpr (m < 4) {
        w_acc = w.w[3];
        if (p.dur_mode) {
          const U4 w1 = philox(it, (uint32_t)f, (uint32_t)s, 1u, p.key0, p.key1);
          kl = 1 + (int)__umulhi(w1.w[1], (uint32_t)K);
        }
      } else {
        const U4 w1 = philox(it, (uint32_t)f, (uint32_t)s, 1u, p.key0, p.key1);
        w_acc = w1.w[0];
        if (p.dur_mode) kl = 1 + (int)__umulhi(w1.w[1], (uint32_t)K);
      }
      // learned proposal: with probability mix_thr / 2^32 the control comes
      // from the network's Gaussian for this frontier entry instead
      if (p.mix_thr != 0ull) {
        const U4 wm = philox(it, (uint32_t)f, (uint32_t)s, 4u, p.key0, p.key1);
        if ((unsigned long long)wm.w[0] < p.mix_thr) {
          const float4 mu = reinterpret_cast<const float4*>(d.head + (size_t)e * 8)[0];
          const float4 sd = reinterpret_cast<const float4*>(d.head + (size_t)e * 8)[1];
          const U4 wz = philox(it, (uint32_t)f, (uint32_t)s, 5u, p.key0, p.key1);
          float z[4];
          box_muller(wz.w[0], wz.w[1], &z[0], &z[1]);
          box_muller(wz.w[2], wz.w[3], &z[2], &z[3]);
          const float mv[4] = {mu.x, mu.y, mu.z, mu.w};
          const float sv[4] = {sd.x, sd.y, sd.z, sd.w};
#pragma unroll
          for (int j = 0; j < m; ++j)
            u[j] = fminf(fmaxf(__builtin_fmaf(sv[j], z[j], mv[j]), p.u_lo[j]), p.u_hi[j]);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < n; ++k) x[k] = 0.0f;
#pragma unroll
      for (int j = 0; j < m; ++j) u[j] = 0.0f;
    }

    // Obstacle culling (without the grid).  Each lane has a reach box that
    // holds every swept box its checked steps can test.  Double integrator:
    // the box of the whole segment's positions (segment_box_di).
    // Quadcopter: until its first failing step a segment stays within rc
    // (per axis) of its parent, since every checked step starts from a state
    // inside the velocity bounds, and near the straight line of its parent's
    // velocity (the accelerations are bounded).  Obstacles that overlap the union of the
    // wave's reach boxes grown by the margin form the wave's union list.  The
    // parents of one tile can lie far apart, and then the union box covers
    // much of the scene; one such tile ran several times longer than the
    // rest and set the launch time.  So a long union list is culled again
    // per group of four lanes (one parent when lambda = 4) into short group
    // lists; a lane tests only its group's list.
    const uint16_t* my = cand;  // this lane's candidate list and its length
    uint32_t mycnt = 0;
    uint32_t kmax = 0;          // every list is read to this even length
    uint32_t ij01 = 0;          // the list's first two entries
    if (!use_grid) {
      const float big = 3.0e38f;
      float rlo[3], rhi[3];
      if constexpr (DYN == KP_DYN_DI6) {
        segment_box_di<INTEG>(x, u, K, sc.h, rlo, rhi);
      } else {
        // An RK4 (or Euler) step moves a position by h v plus a weighted sum
        // of stage accelerations, and the velocity by such a sum, with
        // non-negative weights: after j steps p_j - p_0 - j h v_0 is (j h)^2 / 2
        // times a mean of accelerations, inside [ra_lo, ra_hi] per axis
        // whatever the attitude.  So the positions lie within those offsets
        // of the line from p_0 to p_0 + K h v_0.  The reach box is that,
        // widened by a bound on the FP32 rounding of K steps, and cut to rc.
        const float tk = (float)K * p.h;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float dv = tk * x[6 + a];
          const float eps = 1e-3f + (float)(K + 4) * 1e-6f * (1.0f + fabsf(x[a]) + p.rc);
          rlo[a] = x[a] + fmaxf(fminf(dv, 0.0f) + p.ra_lo[a] - eps, -p.rc);
          rhi[a] = x[a] + fminf(fmaxf(dv, 0.0f) + p.ra_hi[a] + eps, p.rc);
        }
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        rlo[a] = active ? rlo[a] : big;
        rhi[a] = active ? rhi[a] : -big;
      }
      const float bx0 = wave_min(rlo[0]);
      const float by0 = wave_min(rlo[1]);
      const float bz0 = wave_min(rlo[2]);
      const float bx1 = wave_max(rhi[0]);
      const float by1 = wave_max(rhi[1]);
      const float bz1 = wave_max(rhi[2]);
      uint32_t ncand = 0;
      for (int k0 = 0; k0 < n_obs; k0 += 64) {
        const int k = k0 + (int)__lane_id();
        bool ov = false;
        if (k < n_obs) {
          ov = box_separation(bx0 - p.margin, by0 - p.margin, bz0 - p.margin, bx1 + p.margin,
                              by1 + p.margin, bz1 + p.margin, obox + 3 * k) <= 0.0f;
        }
        const unsigned long long b = __ballot(ov);
        if (ov) cand[ncand + __popcll(b & lanes_below())] = (uint16_t)k;
        ncand += (uint32_t)__popcll(b);
      }
      // the candidate lists are private to this wave: order their LDS writes
      // before the reads of other lanes below
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const uint32_t lane = __lane_id();
      mycnt = ncand;
      if (ncand > kGroupCull) {
        // group box: the reach boxes of lanes 4q .. 4q+3
        float q0 = rlo[0], q1 = rlo[1], q2 = rlo[2], q3 = rhi[0], q4 = rhi[1], q5 = rhi[2];
        static_assert(kLaneGroup == 4, "group boxes are reduced inside quads");
        q0 = quad_min(q0);
        q1 = quad_min(q1);
        q2 = quad_min(q2);
        q3 = quad_max(q3);
        q4 = quad_max(q4);
        q5 = quad_max(q5);
        // in the passes below lane l serves group l % 16 and union entries
        // c0 + l / 16, so one pass tests four entries against all 16 groups
        const uint32_t gq = lane & (kGroupsPerWave - 1);
        const int src = (int)gq * kLaneGroup;
        const float mg = p.margin;
        const float b0 = __shfl(q0, src) - mg, b1 = __shfl(q1, src) - mg,
                    b2 = __shfl(q2, src) - mg;
        const float b3 = __shfl(q3, src) + mg, b4 = __shfl(q4, src) + mg,
                    b5 = __shfl(q5, src) + mg;
        const unsigned long long gm = 0x0001000100010001ull << gq;
        uint32_t qn = 0;
        for (uint32_t c0 = 0; c0 < ncand; c0 += 4) {
          const uint32_t ci = c0 + (lane >> 4);
          bool ov = false;
          uint32_t ob = 0;
          if (ci < ncand) {
            ob = cand[ci];
            ov = box_separation(b0, b1, b2, b3, b4, b5, obox + 3 * ob) <= 0.0f;
          }
          const unsigned long long hb = __ballot(ov) & gm;
          const uint32_t pos = qn + (uint32_t)__popcll(hb & lanes_below());
          if (ov && pos < (uint32_t)kGroupCap) glist[gq * kGroupStride + pos] = (uint16_t)ob;
          qn += (uint32_t)__popcll(hb);
        }
        if (lane < (uint32_t)kGroupsPerWave) gcnt[lane] = qn;
        // every group fits: each lane takes its group's list; else the union
        if (__ballot(qn > (uint32_t)kGroupCap) == 0ull) {
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          const uint32_t g4 = lane / kLaneGroup;
          my = glist + g4 * kGroupStride;
          mycnt = gcnt[g4];
        }
      }
      // every list is read to the same even length; pad with the sentinel
      kmax = (wave_max_u32(mycnt) + 1u) & ~1u;
      for (uint32_t k = mycnt + (lane & (kLaneGroup - 1)); k < kmax; k += kLaneGroup)
        const_cast<uint16_t*>(my)[k] = (uint16_t)n_obs;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      ij01 = *reinterpret_cast<const uint32_t*>(my);
    }

    // x' = PropagateODE(x, u, dt): every lane integrates its whole segment.
    // Validity is decided step by step along the way (state box, then the
    // swept box against the candidate obstacles); a lane that fails keeps
    // integrating to its end without further tests, since x' of an invalid
    // sample still decides which region's n_invalid it counts in (Alg. 2).
    YawFrame yf{0.0f, 1.0f, 0.0f, 0.0f};
    if constexpr (DYN == KP_DYN_QUAD12) {
      yf.psi0 = x[5];
      sincos_rr(x[5], &yf.s0, &yf.c0);
    }
    bool alive = active;
    bool valid = active;
    int32_t steps = 0;
    int32_t fstep = 0;   // first failing step (0 while none)
    uint32_t box_tests = 0;
    for (int j = 0; j < K; ++j) {
      if (__ballot(alive) == 0ull) break;
      if (alive) {
        const float px = x[0], py = x[1], pz = x[2];
        integ_step<DYN, INTEG>(sc, x, u, yf);
        steps = j + 1;
        if (valid) {
          bool ok;
          if constexpr (DYN == KP_DYN_QUAD12 && SYM) ok = state_ok_lds_sym(bnd, x);
          else ok = state_ok_lds<DYN>(bnd, x);
          if (ok) {
            const float lx = fminf(px, x[0]) - margin, hx = fmaxf(px, x[0]) + margin;
            const float ly = fminf(py, x[1]) - margin, hy = fmaxf(py, x[1]) + margin;
            const float lz = fminf(pz, x[2]) - margin, hz = fmaxf(pz, x[2]) + margin;
            // closed boxes: touching is a hit.  Each candidate takes the
            // separation form (the same decisions as six comparisons), whose
            // maxima stay on the vector unit instead of joining six lane
            // masks on the scalar unit.
            bool hit = false;
            if (use_grid) {
              // the obstacles listed in the grid cells the swept box touches:
              // its cell range, widened by 1e-3 of a cell so that FP32
              // rounding of the index map cannot drop a cell (the lists were
              // built with the same slack); on one row of cells (fixed y, z)
              // the lists of the x range are contiguous
              const float gi = p.og_inv;
              const int cx0 = clamp_cell((lx - p.og_org[0]) * gi - 1e-3f, gnx);
              const int cx1 = clamp_cell((hx - p.og_org[0]) * gi + 1e-3f, gnx);
              const int cy0 = clamp_cell((ly - p.og_org[1]) * gi - 1e-3f, gny);
              const int cy1 = clamp_cell((hy - p.og_org[1]) * gi + 1e-3f, gny);
              const int cz0 = clamp_cell((lz - p.og_org[2]) * gi - 1e-3f, p.og_n[2]);
              const int cz1 = clamp_cell((hz - p.og_org[2]) * gi + 1e-3f, p.og_n[2]);
              if (__builtin_expect(__ballot(cy1 - cy0 > 1 || cz1 - cz0 > 1) == 0ull, 1)) {
                // A step shorter than a cell touches at most 2 x 2 rows of
                // cells.  Their four entry ranges are read at once, and one
                // flat loop runs over the lane's entries: the wave makes as
                // many trips as its longest list, not one pass per row with
                // every lane waiting for the row's longest list.
                // (every row index is clamped into the range, so the eight
                // offset reads go out together; a row past the range counts 0)
                uint32_t kb[4], kn[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const int cy = min(cy0 + (r & 1), cy1), cz = min(cz0 + (r >> 1), cz1);
                  const int row = (cz * gny + cy) * gnx;
                  kb[r] = goff[row + cx0];
                  const uint32_t ke = goff[row + cx1 + 1];
                  const bool in = cy0 + (r & 1) <= cy1 && cz0 + (r >> 1) <= cz1;
                  kn[r] = in ? ke - kb[r] : 0u;
                }
                const uint32_t c1 = kn[0], c2 = c1 + kn[1], c3 = c2 + kn[2], tn = c3 + kn[3];
                box_tests += tn;
                auto entry = [&](uint32_t t) {
                  return t < c1 ? kb[0] + t
                                : t < c2 ? kb[1] + (t - c1) : t < c3 ? kb[2] + (t - c2) : kb[3] + (t - c3);
                };
                // two entries per trip, so that their LDS reads overlap; past
                // the end the sentinel box n_obs (which nothing touches) stands in
                for (uint32_t t = 0; t < tn; t += 2) {
                  const uint32_t ia = gent[entry(t)];
                  const uint32_t ib = (t + 1 < tn) ? (uint32_t)gent[entry(t + 1)] : (uint32_t)n_obs;
                  const float sa = box_separation(lx, ly, lz, hx, hy, hz, obox + 3 * ia);
                  const float sb = box_separation(lx, ly, lz, hx, hy, hz, obox + 3 * ib);
                  hit |= fminf(sa, sb) <= 0.0f;
                }
              } else {
                for (int cz = cz0; cz <= cz1; ++cz) {
                  for (int cy = cy0; cy <= cy1; ++cy) {
                    const int row = (cz * gny + cy) * gnx;
                    const uint32_t k1 = goff[row + cx1 + 1];
                    uint32_t k = goff[row + cx0];
                    box_tests += k1 - k;
                    for (; k < k1; ++k)
                      hit |= box_separation(lx, ly, lz, hx, hy, hz, obox + 3 * gent[k]) <= 0.0f;
                  }
                }
              }
            } else {
              // two candidates per trip (one 32-bit read of their indices) so
              // that their LDS reads overlap.  The first pair's indices stay
              // in a register for the whole segment, and each trip reads the
              // next pair's together with its own boxes, so a trip waits for
              // one LDS round trip, not two.  (The read past the last pair
              // stays inside this wave's lists: a group list has room for
              // kGroupCap + 2 entries and the union list is followed by the
              // group lists; its value is not used.)
              const uint32_t* my32 = reinterpret_cast<const uint32_t*>(my);
              uint32_t ij = ij01;
              for (uint32_t q = 0; q < kmax; q += 2) {
                const uint32_t ijn = my32[(q >> 1) + 1];
                const float sa = box_separation(lx, ly, lz, hx, hy, hz, obox + 3 * (ij & 0xffffu));
                const float sb = box_separation(lx, ly, lz, hx, hy, hz, obox + 3 * (ij >> 16));
                hit |= fminf(sa, sb) <= 0.0f;
                ij = ijn;
              }
              box_tests += mycnt;
            }
            ok = !hit;
          }
          if (!ok) {
            valid = false;
            fstep = j + 1;
          }
        }
        if (j + 1 == kl) alive = false;  // the segment's duration is over
      }
    }

    // sub-region, n_valid / n_invalid and acceptance (Alg. 2)
    uint32_t cl = 0;
    bool accept = false, goal = false;
    if (active) {
      const bool fin = __builtin_isfinite(x[0]) && __builtin_isfinite(x[1]) &&
                       __builtin_isfinite(x[2]);
      cl = fin ? cell_of(p, x[0], x[1], x[2]) : d.cell[f];
      if (valid) {
        const uint32_t r = cl >> 6;
        // both words are requested before either is used (one round trip)
        const unsigned long long vis = d.visited[r], thr = d.thr[r];
        const bool unvisited = ((vis >> (cl & 63u)) & 1ull) == 0ull;
        accept = unvisited || ((unsigned long long)w_acc < thr);
        const float dx = x[0] - p.goal_c[0], dy = x[1] - p.goal_c[1], dz = x[2] - p.goal_c[2];
        goal = accept && (dx * dx + dy * dy + dz * dz <= p.goal_r2);
        if (goal) c->goal_hit = 1u;
      }
    }
    // n_valid / n_invalid: one atomic per distinct (region, validity) in the wave
    {
      const uint32_t key = active ? ((cl >> 6) << 1) | (valid ? 1u : 0u) : 0xffffffffu;
      unsigned long long pending = __ballot(active);
      while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t k0 = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const unsigned long long match = __ballot(key == k0);
        if ((int)__lane_id() == leader) {
          unsigned long long* ctr = (k0 & 1u) ? d.nv : d.ni;
          atomicAdd(&ctr[k0 >> 1], (unsigned long long)__popcll(match));
        }
        pending &= ~match;
      }
    }

    // Accepted samples are compacted inside the wave's tile (lane order) into
    // the staging area; k_commit later gives them their tree ids.  No wave
    // ever waits for another, so slow tiles do not hold up fast ones.
    const unsigned long long ab = __ballot(accept);
    const uint32_t rank = (uint32_t)__popcll(ab & lanes_below());
    if (accept) {
      const size_t slot = (size_t)tile * 64u + rank;
#pragma unroll
      for (int k = 0; k < n; ++k) d.sx[(size_t)k * d.capP + slot] = x[k];
#pragma unroll
      for (int j = 0; j < m; ++j) d.su[(size_t)j * d.capP + slot] = u[j];
      d.scell[slot] = cl;
      d.slane[slot] = ((uint32_t)g << 1) | (goal ? 1u : 0u);
      d.spar[slot] = f;
    }
    if (__lane_id() == 0) {
      const uint32_t na = (uint32_t)__popcll(ab);
      d.scount[tile] = na;
      if (na) atomicAdd(&ssum_it[tile / kChunkTiles], na);
    }
    const int32_t id = -1;  // assigned by k_commit
    if (trace != nullptr && active) {
      TraceRec* t = trace + g;
      t->parent = f;
      t->sample = s;
#pragma unroll
      for (int j = 0; j < 4; ++j) t->u[j] = (j < m) ? u[j] : 0.0f;
#pragma unroll
      for (int k = 0; k < 12; ++k) t->x[k] = (k < n) ? x[k] : 0.0f;
      t->steps = steps;
      t->fail_step = valid ? steps + 1 : fstep;
      t->valid = valid ? 1 : 0;
      t->cell = cl;
      t->goal = goal ? 1 : 0;
      t->accept = accept ? 1 : 0;
      t->new_id = id;
    }
    // the group's tickets hand out tiles nwaves + grp, nwaves + ng + grp, ...;
    // when the first of them is past the end (a launch with fewer tiles than
    // the grid has waves) the wave is done without the atomic's round trip
    if (nwaves + grp >= ntiles) {
      next = ntiles;
    } else {
      uint32_t tk = 0;
      if (__lane_id() == 0) tk = atomicAdd(&c->tkp[grp].v, 1u);
      next = nwaves + ng * __builtin_amdgcn_readfirstlane(tk) + grp;
    }
    t_lanes += (unsigned long long)__popcll(__ballot(active));
    t_valid += (unsigned long long)__popcll(__ballot(active && valid));
    t_steps += wave_sum_u64((unsigned long long)steps);
    t_checked += wave_sum_u64((unsigned long long)(valid ? steps : fstep));
    t_box += wave_sum_u64((unsigned long long)box_tests);
  }

  __shared__ unsigned long long s_tot[kWaves][5];
  if (__lane_id() == 0) {
    s_tot[wave][0] = t_lanes;
    s_tot[wave][1] = t_valid;
    s_tot[wave][2] = t_steps;
    s_tot[wave][3] = t_box;
    s_tot[wave][4] = t_checked;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long a[5] = {0, 0, 0, 0, 0};
    for (int w = 0; w < kWaves; ++w)
      for (int q = 0; q < 5; ++q) a[q] += s_tot[w][q];
    if (a[0]) {
      TotLine* t = &c->tot[vb % kGroups];
      atomicAdd(&t->lanes, a[0]);
      atomicAdd(&t->valid, a[1]);
      atomicAdd(&t->steps, a[2]);
      atomicAdd(&t->box, a[3]);
      atomicAdd(&t->checked, a[4]);
    }
  }
}

// ---------------------------------------------------------------------------
// k_commit: ids of the accepted samples (V_U of Alg. 2), stable in lane order
// ---------------------------------------------------------------------------
// The V_U scatter of wave tiles first_wt, first_wt + stride, ...: each
// staged sample gets id |T| + (accepted samples of all earlier tiles) +
// (rank inside its tile) and its tree entries.
struct CommitCtx {
  int32_t N, lanes, lam;
  uint32_t it, nwt;
};
__device__ __forceinline__ void commit_tiles(const Params& p, const Dev& d, Ctl* c,
                                             const CommitCtx& k, uint32_t first_wt,
                                             uint32_t stride, TraceRec* trace) {
  const uint32_t lane = __lane_id();
  for (uint32_t wt = first_wt; wt < k.nwt; wt += stride) {
    const uint32_t cnt = d.scount[wt];
    if (cnt == 0u) continue;
    // The staged record and the parent id do not depend on the tile's
    // offset: their loads go out together with the offset's.
    const bool mine = lane < cnt;
    const size_t slot = (size_t)wt * 64u + lane;
    uint32_t sl = 0, scl = 0;
    int32_t par = 0;
    float xs[12], us[4];
    if (mine) {
      sl = d.slane[slot];
      scl = d.scell[slot];
#pragma unroll
      for (int q = 0; q < 12; ++q)
        if (q < p.n) xs[q] = d.sx[(size_t)q * d.capP + slot];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < p.m) us[q] = d.su[(size_t)q * d.capP + slot];
      par = d.spar[slot];
    }
    const uint32_t ch = wt / kChunkTiles;
    unsigned long long part = 0;
    const uint32_t* ssum = d.ssum + (size_t)(k.it & 1u) * (size_t)d.nchunk;
    for (uint32_t j = lane; j < ch; j += 64u) part += ssum[j];
    // the (at most kChunkTiles - 1) earlier counts of the chunk: all loads issued at once
    const uint32_t c0 = ch * kChunkTiles + lane;
#pragma unroll
    for (int q = 0; q < kChunkTiles / 64; ++q) {
      const uint32_t j = c0 + 64u * (uint32_t)q;
      part += (j < wt) ? d.scount[j] : 0u;
    }
    const uint32_t pre = (uint32_t)wave_sum_u64(part);
    if (mine) {
      const int32_t id = k.N + (int32_t)(pre + lane);
      if (id >= k.N + k.lanes) {  // cannot happen with consistent counts; never write past it
        atomicOr(&c->err, 2u);
      } else {
        const int32_t g = (int32_t)(sl >> 1);
        const int32_t s = g - (g / k.lam) * k.lam;
#pragma unroll
        for (int q = 0; q < 12; ++q)
          if (q < p.n) d.x[(size_t)q * d.capP + id] = xs[q];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < p.m) d.u[(size_t)q * d.capP + id] = us[q];
        d.parent[id] = par;
        d.cell[id] = scl;
        d.flag[id] = 1;
        d.birth[id] = (int32_t)k.it;
        d.sample[id] = (uint8_t)s;
        if (sl & 1u) atomicMin(&c->goal_id, id);
        if (trace != nullptr) trace[g].new_id = id;
      }
    }
  }
}

// Each wave takes 64-lane propagate tiles, grid-stride over the waves of the
// commit blocks.  Its staged samples take ids |T| + (accepted samples of all
// earlier tiles) + (rank inside the tile).  The earlier-tile count is the
// sum of the chunk totals before the tile's chunk plus the per-tile counts
// inside it: at most a few loads per lane, with no wait on any other block.
// The first wave of block 0 publishes |V_U| (the sum of all chunk totals)
// and clears the propagate tickets; k_nodesets clears the chunk totals.
// With with_region set, the last block instead runs UpdateEstimates (Alg. 3):
// it reads only what k_propagate wrote and the tree's visited bits, none of
// which the commit blocks touch, so the two run side by side.
template <int NT>
__device__ void region_body(const Env* __restrict__ env);

__global__ __launch_bounds__(kCommitBlock) void k_commit(const Env* __restrict__ env,
                                                         TraceRec* trace, int with_region) {
  if (with_region && blockIdx.x == gridDim.x - 1u) {
    region_body<kCommitBlock>(env);
    return;
  }
  const uint32_t nblk = with_region ? gridDim.x - 1u : gridDim.x;  // >= 1 (launcher)
  const Params& p = env->p;
  const Dev& d = env->d;
  Ctl* c = d.ctl;
  const int done = c->done;
  const int32_t lanes = c->lanes;
  const int32_t lam = c->lambda;
  const int32_t N = c->N;
  const uint32_t it = (uint32_t)c->it;
  const uint32_t nwt = done ? 0u : (uint32_t)((lanes + 63) / 64);  // wave tiles
  const uint32_t lane = __lane_id();
  const uint32_t wave = threadIdx.x >> 6;
  if (blockIdx.x == 0 && wave == 0) {
    const uint32_t nch = (nwt + kChunkTiles - 1) / kChunkTiles;
    unsigned long long part = 0;
    const uint32_t* ssum = d.ssum + (size_t)(it & 1u) * (size_t)d.nchunk;
    for (uint32_t j = lane; j < nch; j += 64u) part += ssum[j];
    part = wave_sum_u64(part);
    if (lane == 0) {
      if (!done) c->nU = (int32_t)part;
      c->sN = N;
      c->snU = done ? 0 : (int32_t)part;
      c->sit = (int32_t)it;
      c->sdone = done;
      c->sepoch = c->epoch;
      c->tk_nodes = 0u;
    }
    if (lane < (uint32_t)kGroups) c->tkp[lane].v = 0u;
  }
  constexpr uint32_t wpb = kCommitBlock / 64;
  CommitCtx k;
  k.N = N;
  k.lanes = lanes;
  k.lam = lam;
  k.it = it;
  k.nwt = nwt;
  commit_tiles(p, d, c, k, blockIdx.x * wpb + wave, nblk * wpb, trace);
}

// ---------------------------------------------------------------------------
// k_region: Alg. 3 (eqs. 3-5), one workgroup
// ---------------------------------------------------------------------------
// Score without the common factor vol^4; fixed FP64 operation order.
__device__ __forceinline__ double region_score(double delta, unsigned long long nv,
                                               unsigned long long ni, int cov) {
  const double a = delta + (double)nv;
  const double b = a + (double)ni;
  const double phi = a / b;
  const double phi2 = phi * phi;
  const double num = phi2 * phi2;
  const double nn = (double)(nv + ni);
  const double den = (1.0 + (double)cov) * (1.0 + nn * nn);
  return num / den;
}

// P_accept = min(1, q / Q + eps) of a region with score sc as a 32-bit
// threshold, the scores scaled by 2^(46 - e) (e: exponent of the largest).
__device__ __forceinline__ unsigned long long region_thr(double sc, int e, unsigned long long Q,
                                                         double eps) {
  const unsigned long long qr = (unsigned long long)floor(ldexp(sc, 46 - e));
  const double P = (Q > 0ull) ? (double)qr / (double)Q + eps : eps;
  return (P >= 1.0) ? (1ull << 32) : (unsigned long long)floor(P * 4294967296.0);
}

// One workgroup of NT threads: three passes over the regions.
// Up to kRegionsHeld regions per thread keep their score in registers
// across the three passes (one read of the region counters); larger grids
// recompute the score in each pass.  Same arithmetic either way.
constexpr int kRegionsHeld = 4;

template <int NT>
__device__ void region_body(const Env* __restrict__ env) {
  const Params& p = env->p;
  const Dev& d = env->d;
  Ctl* c = d.ctl;
  if (c->done) return;
  __shared__ double s_max[NT / 64];
  __shared__ unsigned long long s_sum[NT / 64];
  const int wave = threadIdx.x >> 6;
  const bool held = p.R <= kRegionsHeld * NT;
  double sc_h[kRegionsHeld];
  // pass 1: largest score (a region outside R_avail scores -1)
  double mx = 0.0;
  if (held) {
#pragma unroll
    for (int k = 0; k < kRegionsHeld; ++k) {
      const int r = threadIdx.x + k * NT;
      sc_h[k] = -1.0;
      if (r < p.R && d.avail[r])
        sc_h[k] = region_score(p.delta, d.nv[r], d.ni[r], __popcll(d.visited[r]));
      mx = fmax(mx, sc_h[k]);
    }
  } else {
    for (int r = threadIdx.x; r < p.R; r += NT)
      if (d.avail[r])
        mx = fmax(mx, region_score(p.delta, d.nv[r], d.ni[r], __popcll(d.visited[r])));
  }
  mx = wave_max_f64(mx);
  if (__lane_id() == 0) s_max[wave] = mx;
  __syncthreads();
  mx = 0.0;
  for (int k = 0; k < NT / 64; ++k) mx = fmax(mx, s_max[k]);
  const int e = (mx > 0.0) ? ilogb(mx) : 0;
  // pass 2: exact integer sum of the scores scaled by 2^(46 - e)
  unsigned long long q = 0;
  if (held) {
#pragma unroll
    for (int k = 0; k < kRegionsHeld; ++k)
      if (sc_h[k] >= 0.0) q += (unsigned long long)floor(ldexp(sc_h[k], 46 - e));
  } else {
    for (int r = threadIdx.x; r < p.R; r += NT)
      if (d.avail[r]) {
        const double sc = region_score(p.delta, d.nv[r], d.ni[r], __popcll(d.visited[r]));
        q += (unsigned long long)floor(ldexp(sc, 46 - e));
      }
  }
  q = wave_sum_u64(q);
  if (__lane_id() == 0) s_sum[wave] = q;
  __syncthreads();
  unsigned long long Q = 0;
  for (int k = 0; k < NT / 64; ++k) Q += s_sum[k];
  // pass 3: P_accept = min(1, q / Q + eps) as a 32-bit threshold
  auto thr_of = [&](double sc) { return region_thr(sc, e, Q, p.eps); };
  if (held) {
#pragma unroll
    for (int k = 0; k < kRegionsHeld; ++k) {
      const int r = threadIdx.x + k * NT;
      if (r < p.R && sc_h[k] >= 0.0) d.thr[r] = thr_of(sc_h[k]);
    }
  } else {
    for (int r = threadIdx.x; r < p.R; r += NT) {
      if (!d.avail[r]) continue;
      d.thr[r] = thr_of(region_score(p.delta, d.nv[r], d.ni[r], __popcll(d.visited[r])));
    }
  }
}

__global__ __launch_bounds__(kRegionBlock) void k_region(const Env* __restrict__ env) {
  region_body<kRegionBlock>(env);
}

// Wait until *ctr (incremented once by each region block) reaches n.  Every
// region block of a grid row is dispatched before any other block of that
// row, so they are resident together; the spin is bounded all the same.
__device__ __forceinline__ void wait_count(Ctl* c, uint32_t* ctr, uint32_t n) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n) {
      if (++spins > (1u << 22)) {
        atomicOr(&c->err, 8u);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
  }
  __syncthreads();
}

// UpdateEstimates in k_post, over nrb blocks of NT threads: block b holds
// regions b * kRegionsPerBlock + threadIdx.x + k * NT (k < kRegionsPerBlock / NT) in registers.
// The largest score and the exact sum of the scaled scores are combined
// across the blocks with device atomics (a maximum and an integer sum give
// the same result in any order), so the thresholds are those of the
// one-block pass.  The last block to write its thresholds publishes the
// epoch in region_ready.
template <int NT>
__device__ void region_part(const Env* __restrict__ env, uint32_t b, uint32_t nrb, uint32_t epoch) {
  constexpr int kRT = kRegionsPerBlock / NT;  // regions per thread, held in registers
  static_assert(kRegionsPerBlock == kRT * NT && kRT >= 1, "whole regions per thread");
  const Params& p = env->p;
  const Dev& d = env->d;
  Ctl* c = d.ctl;
  __shared__ double s_max[NT / 64];
  __shared__ unsigned long long s_sum[NT / 64];
  const int wave = threadIdx.x >> 6;
  double sc[kRT];
  double mx = 0.0;
#pragma unroll
  for (int k = 0; k < kRT; ++k) {
    const int r = (int)b * kRegionsPerBlock + threadIdx.x + k * NT;
    sc[k] = -1.0;
    if (r < p.R && d.avail[r])
      sc[k] = region_score(p.delta, d.nv[r], d.ni[r], __popcll(d.visited[r]));
    mx = fmax(mx, sc[k]);
  }
  mx = wave_max_f64(mx);
  if (__lane_id() == 0) s_max[wave] = mx;
  __syncthreads();
  mx = 0.0;
  for (int k = 0; k < NT / 64; ++k) mx = fmax(mx, s_max[k]);
  if (nrb > 1) {
    // non-negative doubles order like their bit patterns
    if (threadIdx.x == 0) {
      atomicMax(&c->rg_max, (unsigned long long)__double_as_longlong(mx));
      __threadfence();
      atomicAdd(&c->rg_cnt_max, 1u);
    }
    wait_count(c, &c->rg_cnt_max, nrb);
    mx = __longlong_as_double((long long)__hip_atomic_load(&c->rg_max, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT));
  }
  const int e = (mx > 0.0) ? ilogb(mx) : 0;
  unsigned long long q = 0;
#pragma unroll
  for (int k = 0; k < kRT; ++k)
    if (sc[k] >= 0.0) q += (unsigned long long)floor(ldexp(sc[k], 46 - e));
  q = wave_sum_u64(q);
  if (__lane_id() == 0) s_sum[wave] = q;
  __syncthreads();
  unsigned long long Q = 0;
  for (int k = 0; k < NT / 64; ++k) Q += s_sum[k];
  if (nrb > 1) {
    if (threadIdx.x == 0) {
      atomicAdd(&c->rg_sum, Q);
      __threadfence();
      atomicAdd(&c->rg_cnt_sum, 1u);
    }
    wait_count(c, &c->rg_cnt_sum, nrb);
    Q = __hip_atomic_load(&c->rg_sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
#pragma unroll
  for (int k = 0; k < kRT; ++k) {
    const int r = (int)b * kRegionsPerBlock + threadIdx.x + k * NT;
    if (r < p.R && sc[k] >= 0.0) d.thr[r] = region_thr(sc[k], e, Q, p.eps);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t prev = (nrb > 1) ? atomicAdd(&c->rg_cnt_thr, 1u) : 0u;
    if (prev + 1u == nrb)
      __hip_atomic_store(&c->region_ready, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// k_nodesets: Alg. 4 + next frontier + eq. (6)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kNodeBlock) void k_nodesets(const Env* __restrict__ env) {
  const Params& p = env->p;
  const Dev& d = env->d;
  Ctl* c = d.ctl;
  const int done = c->sdone;
  const int32_t N = c->sN;
  const int32_t nU = c->snU;
  const int32_t Nt = N + nU;
  const uint32_t it = (uint32_t)c->sit;
  const uint32_t epoch = c->sepoch;
  const bool goal = c->goal_id != kNoGoal;
  const uint32_t ntiles = done ? 0u : (uint32_t)((Nt + kNodeTile - 1) / kNodeTile);
  // accepted-sample chunk totals of this iteration's expansion: used up
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < 2 * d.nchunk; j += kNodeBlock) d.ssum[j] = 0u;
  // With a tile for every block, tile = block index: blocks start in index
  // order, so a tile's look-back only waits on blocks that started earlier.
  // With more tiles than blocks, every tile comes from the ticket counter
  // (including the first): a block then only waits on tiles handed out
  // before its own, all held by running blocks, whatever the number of
  // blocks that fit on the device at once.  The block that holds the last
  // tile finalises the iteration once its look-back has given the total.
  __shared__ uint32_t s_tile, s_pref, s_wt[kNodeBlock / 64];
  const bool by_ticket = ntiles > gridDim.x;
  uint32_t tile = blockIdx.x;
  if (by_ticket) {
    if (threadIdx.x == 0) s_tile = atomicAdd(&c->tk_nodes, 1u);
    __syncthreads();
    tile = s_tile;
    __syncthreads();
  }
  for (;;) {
    if (tile >= ntiles) break;
    const uint32_t base = tile * kNodeTile + threadIdx.x * kNodesPerThread;
    uint32_t eb = 0;
    // visited bits of new nodes, merged over runs of nodes in one region
    uint32_t run_r = 0xffffffffu;
    unsigned long long run_m = 0ull;
    if (base < (uint32_t)Nt) {
      uint32_t fw[kFlagWords], nfw[kFlagWords];
      load_flag_words(d.flag + base, fw);
#pragma unroll
      for (int q = 0; q < kFlagWords; ++q) nfw[q] = fw[q];
#pragma unroll
      for (int q = 0; q < kNodesPerThread / 4; ++q) {
        const uint32_t b4 = base + 4u * q;
        if (b4 >= (uint32_t)Nt) break;
        const uint4 cw = *reinterpret_cast<const uint4*>(d.cell + b4);
        const uint32_t cells[4] = {cw.x, cw.y, cw.z, cw.w};
        // node pair (2k, 2k+1) shares Philox block (it, k, 0, 3)
        const U4 wa = philox(it, b4 >> 1, 0u, 3u, p.key0, p.key1);
        const U4 wb = philox(it, (b4 >> 1) + 1u, 0u, 3u, p.key0, p.key1);
        const uint32_t wd[4] = {wa.w[0], wa.w[2], wb.w[0], wb.w[2]};
        const uint32_t wp[4] = {wa.w[1], wa.w[3], wb.w[1], wb.w[3]};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t i = b4 + k;
          if (i >= (uint32_t)Nt) continue;
          const uint32_t r = cells[k] >> 6;
          bool E;
          if (i >= (uint32_t)N) {
            // V_U joins T and V_E (Alg. 4)
            E = true;
            if (r != run_r) {
              if (run_m) {
                atomicOr(&d.visited[run_r], run_m);
                d.avail[run_r] = 1;
              }
              run_r = r;
              run_m = 0ull;
            }
            run_m |= 1ull << (cells[k] & 63u);
          } else {
            const unsigned long long t = d.thr[r];
            const bool wasE = ((fw[q] >> (8 * k)) & 0xffu) != 0u;
            const bool stay = wasE && ((unsigned long long)wd[k] < t);   // V_E -> V_O w.p. 1-P
            E = stay || (!goal && ((unsigned long long)wp[k] < t));      // V_O -> V_E w.p. P
            nfw[q] = (nfw[q] & ~(0xffu << (8 * k))) | ((E ? 1u : 0u) << (8 * k));
          }
          if (E) eb |= 1u << (4 * q + k);
        }
      }
      bool changed = false;
#pragma unroll
      for (int q = 0; q < kFlagWords; ++q) changed |= nfw[q] != fw[q];
      if (changed) store_flag_words(d.flag + base, nfw);
      if (run_m) {
        atomicOr(&d.visited[run_r], run_m);
        d.avail[run_r] = 1;
      }
    }
    const uint32_t upto = compact_frontier(d, d.st_nodes, eb, base, tile, epoch, s_wt, &s_pref);
    if (tile == ntiles - 1u && threadIdx.x == 0) {
      c->N = Nt;
      if (goal) c->done = KP_SOLVED;
      finalize_frontier(p, c, upto, Nt);
      c->it = (int32_t)it + 1;
      c->epoch = epoch + 1u;
      c->iters_done += 1u;
    }
    if (!by_ticket) break;
    if (threadIdx.x == 0) s_tile = atomicAdd(&c->tk_nodes, 1u);
    __syncthreads();
    tile = s_tile;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k_post: the rest of a kp_plan iteration after k_propagate, in one launch
// ---------------------------------------------------------------------------
//   block 0            UpdateEstimates (Alg. 3), then publishes region_ready
//   blocks 1 .. nc     V_U: ids and tree entries (commit_tiles); once the
//                      thresholds are out, the new nodes' visited bits and
//                      R_avail (Alg. 4: V_U joins T)
//   blocks nc+1 ..     UpdateNodeSets (Alg. 4) over the old nodes [0, N):
//                      demote / promote once the thresholds are out, and
//                      the compaction of their E flags into F
//   last old tile      its block, once its look-back has the count of old E
//                      nodes: |T| += |V_U|; the frontier is the old E nodes
//                      (F) followed by the new ids N .. N + |V_U| - 1 (all
//                      E, kept implicit); eq. (6); next iteration
// Blocks wait only on block 0, which starts first and waits on nothing, and
// on look-backs ordered as in k_nodesets.  Every block reads the sizes from
// the copy k_propagate made, so the finaliser may run while late blocks
// start.  Same results as k_commit, k_region and k_nodesets in sequence.
// The commit takes each sample's parent from its staged record, never from
// F, which the node-set blocks rewrite in the same launch.
// Thread 0 polls with relaxed device-scope loads.  No acquire fence follows
// (on this GPU it would invalidate the cache of every wave of every waiting
// block): the thresholds are then read with device-scope atomic loads, which
// see the region block's writes once it has published the flag after its
// own device-scope fence.
__device__ __forceinline__ void wait_region(Ctl* c, uint32_t epoch) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (__hip_atomic_load(&c->region_ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
           epoch) {
      if (++spins > (1u << 22)) {
        atomicOr(&c->err, 8u);
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
  }
  __syncthreads();
}

// ---- node-set pass of k_post (Alg. 4) ----
// A thread's four consecutive old nodes: flag bytes, cells and the two
// Philox words of each node (demotion draw wd, promotion draw wp).
struct NodeWords {
  uint32_t fw;
  uint32_t cell[4];
  uint32_t wd[4], wp[4];
};
__device__ __forceinline__ void node_fetch(const Dev& d, uint32_t base, int32_t N, NodeWords* w) {
  w->fw = 0u;
  w->cell[0] = w->cell[1] = w->cell[2] = w->cell[3] = 0u;
  if (base >= (uint32_t)N) return;
  uint32_t f[kFlagWords];
  load_flag_words(d.flag + base, f);
  w->fw = f[0];
  const uint4 cw = *reinterpret_cast<const uint4*>(d.cell + base);
  w->cell[0] = cw.x;
  w->cell[1] = cw.y;
  w->cell[2] = cw.z;
  w->cell[3] = cw.w;
}
__device__ __forceinline__ void node_draws(const Params& p, uint32_t it, uint32_t base, int32_t N,
                                           NodeWords* w) {
  if (base >= (uint32_t)N) return;
  // node pair (2k, 2k+1) shares Philox block (it, k, 0, 3)
  const U4 wa = philox(it, base >> 1, 0u, 3u, p.key0, p.key1);
  const U4 wb = philox(it, (base >> 1) + 1u, 0u, 3u, p.key0, p.key1);
  w->wd[0] = wa.w[0];
  w->wd[1] = wa.w[2];
  w->wd[2] = wb.w[0];
  w->wd[3] = wb.w[2];
  w->wp[0] = wa.w[1];
  w->wp[1] = wa.w[3];
  w->wp[2] = wb.w[1];
  w->wp[3] = wb.w[3];
}
// New V_E membership of the four nodes from their region thresholds (read
// once the region pass has published them); changed flags are written
// back.  Returns the V_E bits.
__device__ __forceinline__ uint32_t node_decide(const Dev& d, uint32_t base, int32_t N, bool goal,
                                                const NodeWords& w) {
  if (base >= (uint32_t)N) return 0u;
  uint32_t nfw = w.fw, eb = 0u;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k >= (uint32_t)N) continue;
    const unsigned long long t = __hip_atomic_load(&d.thr[w.cell[k] >> 6], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
    const bool wasE = ((w.fw >> (8 * k)) & 0xffu) != 0u;
    const bool stay = wasE && ((unsigned long long)w.wd[k] < t);          // V_E -> V_O w.p. 1-P
    const bool E = stay || (!goal && ((unsigned long long)w.wp[k] < t));  // V_O -> V_E w.p. P
    nfw = (nfw & ~(0xffu << (8 * k))) | ((E ? 1u : 0u) << (8 * k));
    if (E) eb |= 1u << k;
  }
  if (nfw != w.fw) {
    if (base + 4u <= (uint32_t)N) {
      store_flag_words(d.flag + base, &nfw);
    } else {
      // the word reaches into V_U, whose flags the commit blocks write
      for (uint32_t k = 0; base + k < (uint32_t)N; ++k)
        d.flag[base + k] = (uint8_t)((nfw >> (8 * k)) & 0xffu);
    }
  }
  return eb;
}
// End of an iteration, by wave 0 of the block that knows the whole old-node
// count of the next frontier (upto, the same in every lane): |V_U| from the
// chunk totals (one load per lane), then lane 0 sets the sizes, eq. (6).
__device__ __forceinline__ void node_finalize(const Params& p, Ctl* c, int32_t N, uint32_t it,
                                              uint32_t epoch, uint32_t nwt, const uint32_t* ssum,
                                              bool goal, uint32_t upto) {
  const uint32_t nch = (nwt + kChunkTiles - 1) / kChunkTiles;
  unsigned long long part = 0;
  for (uint32_t j = __lane_id(); j < nch; j += 64u) part += ssum[j];
  const uint32_t nU = (uint32_t)wave_sum_u64(part);
  if (__lane_id() != 0) return;
  const int32_t Nt = N + (int32_t)nU;
  c->nU = (int32_t)nU;
  c->N = Nt;
  if (goal) c->done = KP_SOLVED;
  finalize_frontier(p, c, upto + nU, Nt);
  c->f_expl = (int32_t)upto;
  c->f_base = N;
  c->it = (int32_t)it + 1;
  c->epoch = epoch + 1u;
  c->iters_done += 1u;
}

// Node sets over a contiguous chunk of `per` tiles (2 .. kChunkTilesMax) per
// block, with no tile tickets (same-address atomics serialise) and one
// look-back per chunk.  Chunk indices follow node order and a lower chunk
// belongs to a block dispatched earlier, so every wait ends whatever the
// number of blocks resident at once.  Pass 1 decides every node of the
// chunk and keeps the thread's V_E bits (4 per tile) in one register; the
// chunk's count gets its global offset from the look-back; pass 2 writes
// the frontier entries tile by tile, in node order.
__device__ __forceinline__ void node_chunk(const Params& p, const Dev& d, Ctl* c, uint32_t bi,
                                           uint32_t per, uint32_t ntiles, int32_t N, uint32_t it,
                                           uint32_t epoch, uint32_t nwt, const uint32_t* ssum,
                                           bool goal, uint32_t* s_wt, uint32_t* s_pref) {
  const uint32_t t0 = bi * per;
  if (t0 >= ntiles) return;
  const uint32_t t1 = (t0 + per < ntiles) ? t0 + per : ntiles;
  const uint32_t lb = threadIdx.x * kNodesPerThread;
  const uint32_t lane = __lane_id();
  const uint32_t wave = threadIdx.x >> 6;
  unsigned long long ebits = 0ull;
  for (uint32_t tile = t0; tile < t1; ++tile) {
    const uint32_t base = tile * kNodeTile + lb;
    NodeWords w;
    node_fetch(d, base, N, &w);
    node_draws(p, it, base, N, &w);
    if (tile == t0) wait_region(c, epoch);
    const uint32_t eb = node_decide(d, base, N, goal, w);
    ebits |= (unsigned long long)eb << (4u * (tile - t0));
  }
  // the chunk's count and its global offset
  const unsigned long long ws = wave_sum_u64((unsigned long long)__popcll(ebits));
  if (lane == 0) s_wt[wave] = (uint32_t)ws;
  __syncthreads();
  uint32_t agg = 0;
#pragma unroll
  for (int k = 0; k < kNodeBlock / 64; ++k) agg += s_wt[k];
  if (wave == 0) {
    const uint32_t pre = lookback_prefix_wave(d.st_nodes, bi, agg, epoch, &c->err, 4u);
    if (lane == 0) *s_pref = pre;
  }
  __syncthreads();
  const uint32_t P = *s_pref;
  uint32_t acc = 0;
  for (uint32_t tile = t0; tile < t1; ++tile) {
    uint32_t eb = (uint32_t)(ebits >> (4u * (tile - t0))) & 0xfu;
    uint32_t wt;
    const uint32_t ex = wave_excl_small((uint32_t)__popc(eb), &wt);
    if (lane == 0) s_wt[wave] = wt;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kNodeBlock / 64; ++k) {
      const uint32_t t = s_wt[k];
      off += ((uint32_t)k < wave) ? t : 0u;
      tot += t;
    }
    __syncthreads();
    uint32_t pos = P + acc + off + ex;
    const uint32_t base = tile * kNodeTile + lb;
    while (eb) {
      const int k = __ffs(eb) - 1;
      d.F[pos++] = (int32_t)(base + k);
      eb &= eb - 1u;
    }
    acc += tot;
  }
  if (t1 == ntiles && threadIdx.x < 64u) node_finalize(p, c, N, it, epoch, nwt, ssum, goal, P + agg);
}

// One post launch's work for block vb of a grid row of vg blocks: nrb
// region blocks, nc commit blocks, then node-set blocks.  solo: one
// workgroup plays the three roles in turn (vb = 0, 1, 2 of vg = 3, nc = 1),
// with a one-block region pass over every region.
__device__ __forceinline__ void post_body(const Env* __restrict__ env, int nc, uint32_t vb,
                                          uint32_t vg, bool solo) {
  static_assert(kCommitBlock == kNodeBlock, "one block shape for every role");
  static_assert(kNodesPerThread == 4, "one flag word and one uint4 of cells per thread");
  const Params& p = env->p;
  const Dev& d = env->d;
  Ctl* c = d.ctl;
  // sizes from k_propagate's copy: the finaliser below rewrites the live ones
  const int done = c->sdone;
  const int32_t N = c->sN;
  const int32_t lanes = c->slanes;
  const int32_t lam = c->slam;
  const uint32_t it = (uint32_t)c->sit;
  const uint32_t epoch = c->sepoch;
  const uint32_t nwt = done ? 0u : (uint32_t)((lanes + 63) / 64);
  const uint32_t* ssum = d.ssum + (size_t)(it & 1u) * (size_t)d.nchunk;
  const uint32_t lane = __lane_id();
  const uint32_t wave = threadIdx.x >> 6;
  constexpr uint32_t wpb = kCommitBlock / 64;
  __shared__ uint32_t s_pref, s_wt[kNodeBlock / 64];

  // grid row: nrb region blocks, the node-set blocks, then nc commit blocks
  // (solo: region, commit, node-set).  The node-set blocks carry the
  // iteration's end, so they are dispatched right after the region blocks;
  // the commit blocks only have to finish before the launch does.
  const uint32_t nrb = solo ? 1u : (uint32_t)post_region_blocks(p.R);
  const uint32_t nb = vg - nrb - (uint32_t)nc;
  const bool commit_role = solo ? vb == 1u : vb >= nrb + nb;
  const uint32_t bi = solo ? 0u : vb - nrb;
  if (vb < nrb) {
    // ---- UpdateEstimates; and the counters of the next expansion ----
    if (vb == 0) {
      uint32_t* nxt = d.ssum + (size_t)((it + 1u) & 1u) * (size_t)d.nchunk;
      for (int j = threadIdx.x; j < d.nchunk; j += kCommitBlock) nxt[j] = 0u;
      if (threadIdx.x < (unsigned)kGroups) c->tkp[threadIdx.x].v = 0u;
    }
    if (!done && !solo) {
      region_part<kCommitBlock>(env, vb, nrb, epoch);
    } else if (vb == 0) {
      if (!done) region_body<kCommitBlock>(env);
      __syncthreads();
      if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_store(&c->region_ready, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    return;
  }
  if (commit_role) {
    const uint32_t ci = solo ? 0u : vb - nrb - nb;
    // ---- V_U ----
    CommitCtx k;
    k.N = N;
    k.lanes = lanes;
    k.lam = lam;
    k.it = it;
    k.nwt = nwt;
    const uint32_t first = ci * wpb + wave, stride = (uint32_t)nc * wpb;
    commit_tiles(p, d, c, k, first, stride, nullptr);
    // visited bits of the block's samples, once the estimates have read the
    // old ones: one atomic per distinct region among a tile's samples.  A
    // block with no accepted sample does not wait.
    bool any = false;
    for (uint32_t wt = ci * wpb; wt < nwt && !any; wt += stride)
      for (uint32_t w = 0; w < wpb && wt + w < nwt; ++w) any |= d.scount[wt + w] != 0u;
    if (!any) return;
    wait_region(c, epoch);
    for (uint32_t wt = first; wt < nwt; wt += stride) {
      const uint32_t cnt = d.scount[wt];
      if (cnt == 0u) continue;
      const uint32_t cl = (lane < cnt) ? d.scell[(size_t)wt * 64u + lane] : 0u;
      const uint32_t key = (lane < cnt) ? (cl >> 6) : 0xffffffffu;
      unsigned long long pending = __ballot(lane < cnt);
      while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const unsigned long long match = __ballot(key == r0);
        const unsigned long long bits = wave_or_u64((key == r0) ? (1ull << (cl & 63u)) : 0ull);
        if ((int)lane == leader) {
          atomicOr(&d.visited[r0], bits);
          d.avail[r0] = 1;
        }
        pending &= ~match;
      }
    }
    return;
  }
  // ---- UpdateNodeSets over the old nodes ----
  const bool goal = c->goal_hit != 0u;
  const uint32_t ntiles = done ? 0u : (uint32_t)((N + kNodeTile - 1) / kNodeTile);
  if (solo) {
    // one workgroup: the chunks one after the other
    for (uint32_t k = 0; k * (uint32_t)kChunkTilesMax < ntiles; ++k)
      node_chunk(p, d, c, k, kChunkTilesMax, ntiles, N, it, epoch, nwt, ssum, goal, s_wt, &s_pref);
    return;
  }
  // the launcher gives at least one node-set block per kChunkTilesMax tiles
  // of its bound on |T|; a grid that breaks this is refused (error bit 16)
  const uint32_t per = (ntiles + nb - 1) / nb;
  if (per > (uint32_t)kChunkTilesMax) {
    if (bi == 0 && threadIdx.x == 0) atomicOr(&c->err, 16u);
    return;
  }
  if (per > 1u) {
    node_chunk(p, d, c, bi, per, ntiles, N, it, epoch, nwt, ssum, goal, s_wt, &s_pref);
    return;
  }
  // one tile per block: tile = block index
  const uint32_t tile = bi;
  if (tile >= ntiles) return;
  const uint32_t base = tile * kNodeTile + threadIdx.x * kNodesPerThread;
  NodeWords w;
  node_fetch(d, base, N, &w);
  node_draws(p, it, base, N, &w);
  wait_region(c, epoch);
  const uint32_t eb = node_decide(d, base, N, goal, w);
  const uint32_t upto = compact_frontier(d, d.st_nodes, eb, base, tile, epoch, s_wt, &s_pref);
  if (tile == ntiles - 1u && threadIdx.x < 64u) node_finalize(p, c, N, it, epoch, nwt, ssum, goal, upto);
}

// One problem per launch, or one problem per grid row (blockIdx.y) of a
// batched launch over a table of problems; the work of each problem is the
// same either way.  Waves per SIMD: 4 (at most 128 registers; one 16-wave
// block per compute unit).  The quadcopter kernels need more than 96 (the
// tilt sin / cos keep their range-checked reduction for segments that have
// left the state box).
template <int DYN, int INTEG, bool SYM>
__global__ __launch_bounds__(prop_block(DYN)) __attribute__((amdgpu_waves_per_eu(4))) void k_propagate(
    const Env* __restrict__ env, TraceRec* trace) {
  propagate_body<DYN, INTEG, SYM, prop_block(DYN)>(env, trace, blockIdx.x, gridDim.x);
}
template <int DYN, int INTEG, bool SYM>
__global__ __launch_bounds__(prop_block(DYN)) __attribute__((amdgpu_waves_per_eu(4))) void k_propagate_batch(
    const Env* const* __restrict__ envs) {
  const Env* env = envs[blockIdx.y];
  propagate_body<DYN, INTEG, SYM, prop_block(DYN)>(env, env->d.trace, blockIdx.x, gridDim.x);
}

// Waves per SIMD: 8 (at most 64 registers), so two 16-wave blocks share a
// compute unit: the node-set blocks of a wide tree are twice as many, and a
// launch's commit blocks do not fill the device on their own.  The batched
// kernel keeps its default (at 64 registers it would spill).
__global__ __launch_bounds__(kCommitBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_post(
    const Env* __restrict__ env, int nc) {
  post_body(env, nc, blockIdx.x, gridDim.x, false);
}
__global__ __launch_bounds__(kCommitBlock) void k_post_batch(const Env* const* __restrict__ envs,
                                                             int nc) {
  post_body(envs[blockIdx.y], nc, blockIdx.x, gridDim.x, false);
}

// compact status of every problem of a batch, for one host read

// ---------------------------------------------------------------------------
// k_plan_queue: batched planning in one launch over a device work queue.
// Each workgroup takes the next problem (order[q] for q = 0, 1, ... from the
// queue head) and runs Alg. 1's loop for it until it stops: goal, full tree
// or empty frontier (done), its iteration budget, or its time budget on the
// device wall clock.  One iteration is the propagate body, then the region
// pass, the V_U commit and the node-set pass, one after the other, with one
// workgroup playing every block of the two-launch grids; the kernels' results
// do not depend on grid shapes, so each problem ends exactly as kp_plan
// leaves it.  Between phases every wave fences at device scope (the phases
// read what device-scope atomics of the previous one wrote) and the
// workgroup synchronises.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void queue_phase_end() {
  __threadfence();
  __syncthreads();
}

template <int DYN, int INTEG, bool SYM>
__global__ __launch_bounds__(kQueueBlock) void k_plan_queue(
    const Env* const* __restrict__ envs, const int32_t* __restrict__ order,
    const QueueJob* __restrict__ jobs, int n, QueueCtl* qc, unsigned long long* __restrict__ t_end,
    int32_t* __restrict__ ran) {
  __shared__ int s_q, s_go;
  if (threadIdx.x == 0) atomicMin(&qc->t_start, (unsigned long long)wall_clock64());
  for (;;) {
    if (threadIdx.x == 0) s_q = (int)atomicAdd(&qc->head, 1u);
    __syncthreads();
    const int q = s_q;
    __syncthreads();
    if (q >= n) return;
    const int i = order[q];
    const Env* env = envs[i];
    Ctl* c = env->d.ctl;
    const int32_t iters = jobs[i].iters;
    const unsigned long long ticks = jobs[i].ticks;
    const unsigned long long t0 = (unsigned long long)wall_clock64();
    int32_t k = 0;
    for (;;) {
      if (threadIdx.x == 0) {
        // done is written by this workgroup's thread 0 (the node pass's finaliser)
        bool go = k < iters && c->done == 0;
        if (go && ticks != 0ull && (unsigned long long)wall_clock64() - t0 >= ticks) go = false;
        s_go = go ? 1 : 0;
      }
      __syncthreads();
      if (!s_go) break;
      propagate_body<DYN, INTEG, SYM, kQueueBlock>(env, env->d.trace, 0u, 1u);
      queue_phase_end();
      for (uint32_t role = 0; role < 3u; ++role) {
        post_body(env, 1, role, 3u, true);
        queue_phase_end();
      }
      ++k;
    }
    if (threadIdx.x == 0) {
      ran[i] = k;
      t_end[i] = (unsigned long long)wall_clock64();
    }
  }
}

__global__ void k_batch_status(const Env* const* __restrict__ envs, int n, BatchStatus* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Ctl* c = envs[i]->d.ctl;
  BatchStatus s;
  s.done = c->done;
  s.N = c->N;
  s.nF = c->nF;
  s.lanes = c->lanes;
  s.iters_done = (int32_t)c->iters_done;
  s.goal_id = c->goal_id;
  s.err = (int32_t)c->err;
  s.pad = 0;
  unsigned long long l = 0, v = 0;
  for (int g = 0; g < kGroups; ++g) {
    l += c->tot[g].lanes;
    v += c->tot[g].valid;
  }
  s.lanes_total = l;
  s.valid_total = v;
  out[i] = s;
}

// ends (code > 0) or resumes (code 0) a problem's iterations: every kernel of
// an iteration returns at once while done != 0
__global__ void k_set_done(const Env* __restrict__ env, int32_t code) {
  if (blockIdx.x == 0 && threadIdx.x == 0) env->d.ctl->done = code;
}

// ---------------------------------------------------------------------------
// k_path: root-to-node walk along parent links
// ---------------------------------------------------------------------------
__global__ void k_path(const Env* __restrict__ env, int32_t node) {
  const Dev& d = env->d;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int32_t len = 0;
  for (int32_t v = node; v >= 0 && len <= kMaxPath; v = d.parent[v]) ++len;
  d.path[0] = len;
  if (len > kMaxPath) return;
  int32_t k = len;
  for (int32_t v = node; v >= 0; v = d.parent[v]) d.path[k--] = v;
}

// Rows of the trajectory along the path k_path wrote: row i holds the state
// of path node i (12 floats), the control of the edge into it (4 floats) and
// that edge's integration steps (as an int), 17 words, in `out`.
constexpr int kTrajWords = 17;
__global__ void k_path_gather(const Env* __restrict__ env, int32_t len, float* __restrict__ out) {
  const Params& p = env->p;
  const Dev& d = env->d;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const int32_t v = d.path[1 + i];
  float* r = out + (size_t)i * kTrajWords;
  for (int k = 0; k < 12; ++k) r[k] = (k < p.n) ? d.x[(size_t)k * d.capP + v] : 0.0f;
  for (int j = 0; j < 4; ++j) r[12 + j] = (j < p.m) ? d.u[(size_t)j * d.capP + v] : 0.0f;
  int32_t ks = 0;
  const int32_t par = d.parent[v];
  if (par >= 0) {
    ks = p.K;
    if (p.dur_mode) {
      const U4 w1 = philox((uint32_t)d.birth[v], (uint32_t)par, (uint32_t)d.sample[v], 1u, p.key0,
                           p.key1);
      ks = 1 + (int32_t)__umulhi(w1.w[1], (uint32_t)p.K);
    }
  }
  r[16] = __int_as_float(ks);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_zero(const Params& p, const Dev& d, const Env* env, hipStream_t s) {
  int work = p.R;
  if (d.tiles_node > work) work = d.tiles_node;
  if (d.nchunk > work) work = d.nchunk;
  int grid = (work + 255) / 256;
  if (grid > 1024) grid = 1024;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, env);
  return hipGetLastError();
}

hipError_t launch_root(const Env* env, Vec12 xi, hipStream_t s) {
  hipLaunchKernelGGL(k_root, dim3(1), dim3(64), 0, s, env, xi);
  return hipGetLastError();
}

hipError_t launch_set_ctl(const Env* env, int32_t N, int32_t it, hipStream_t s) {
  hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, s, env, N, it);
  return hipGetLastError();
}

hipError_t launch_frontier(const Env* env, int grid, hipStream_t s, Timing t) {
  hipExtLaunchKernelGGL(k_frontier, dim3(grid), dim3(kNodeBlock), 0, s, t.start, t.stop, 0, env);
  return hipGetLastError();
}

template <int DYN, int INTEG, bool SYM>
static hipError_t launch_prop_t(const Env* env, size_t lds, TraceRec* trace, int grid,
                                hipStream_t s, Timing t) {
  hipExtLaunchKernelGGL((k_propagate<DYN, INTEG, SYM>), dim3(grid), dim3(prop_block(DYN)),
                        (uint32_t)lds, s, t.start, t.stop, 0, env, trace);
  return hipGetLastError();
}

hipError_t launch_propagate(int dyn, int integ, int sym, const Env* env, size_t lds,
                            TraceRec* trace, int grid, hipStream_t s, Timing t) {
  if (dyn == KP_DYN_DI6 && integ == KP_INT_EULER)
    return launch_prop_t<KP_DYN_DI6, KP_INT_EULER, false>(env, lds, trace, grid, s, t);
  if (dyn == KP_DYN_DI6 && integ == KP_INT_RK4)
    return launch_prop_t<KP_DYN_DI6, KP_INT_RK4, false>(env, lds, trace, grid, s, t);
  if (integ == KP_INT_EULER)
    return sym ? launch_prop_t<KP_DYN_QUAD12, KP_INT_EULER, true>(env, lds, trace, grid, s, t)
                : launch_prop_t<KP_DYN_QUAD12, KP_INT_EULER, false>(env, lds, trace, grid, s, t);
  return sym ? launch_prop_t<KP_DYN_QUAD12, KP_INT_RK4, true>(env, lds, trace, grid, s, t)
              : launch_prop_t<KP_DYN_QUAD12, KP_INT_RK4, false>(env, lds, trace, grid, s, t);
}

hipError_t launch_commit(const Env* env, TraceRec* trace, int grid, int with_region,
                         hipStream_t s, Timing t) {
  if (grid < 1) grid = 1;
  if (with_region) grid += 1;  // the extra, last block runs the region pass
  hipExtLaunchKernelGGL(k_commit, dim3(grid), dim3(kCommitBlock), 0, s, t.start, t.stop, 0, env,
                        trace, with_region);
  return hipGetLastError();
}

hipError_t launch_post(const Env* env, int n_region, int n_commit, int n_nodes, hipStream_t s,
                       Timing t) {
  if (n_commit < 1) n_commit = 1;
  if (n_nodes < 1) n_nodes = 1;
  hipExtLaunchKernelGGL(k_post, dim3(n_region + n_commit + n_nodes), dim3(kCommitBlock), 0, s,
                        t.start, t.stop, 0, env, n_commit);
  return hipGetLastError();
}

hipError_t launch_region(const Env* env, hipStream_t s, Timing t) {
  hipExtLaunchKernelGGL(k_region, dim3(1), dim3(kRegionBlock), 0, s, t.start, t.stop, 0, env);
  return hipGetLastError();
}

hipError_t launch_nodesets(const Env* env, int grid, hipStream_t s, Timing t) {
  hipExtLaunchKernelGGL(k_nodesets, dim3(grid), dim3(kNodeBlock), 0, s, t.start, t.stop, 0, env);
  return hipGetLastError();
}

template <int DYN, int INTEG, bool SYM>
static hipError_t launch_prop_batch_t(const Env* const* envs, int n, size_t lds, int grid,
                                      hipStream_t s) {
  hipLaunchKernelGGL((k_propagate_batch<DYN, INTEG, SYM>), dim3(grid, n), dim3(prop_block(DYN)),
                     (uint32_t)lds, s, envs);
  return hipGetLastError();
}

hipError_t launch_propagate_batch(int dyn, int integ, int sym, const Env* const* envs, int n,
                                  size_t lds, int grid, hipStream_t s) {
  if (grid < 1) grid = 1;
  if (dyn == KP_DYN_DI6 && integ == KP_INT_EULER)
    return launch_prop_batch_t<KP_DYN_DI6, KP_INT_EULER, false>(envs, n, lds, grid, s);
  if (dyn == KP_DYN_DI6 && integ == KP_INT_RK4)
    return launch_prop_batch_t<KP_DYN_DI6, KP_INT_RK4, false>(envs, n, lds, grid, s);
  if (integ == KP_INT_EULER)
    return sym ? launch_prop_batch_t<KP_DYN_QUAD12, KP_INT_EULER, true>(envs, n, lds, grid, s)
                : launch_prop_batch_t<KP_DYN_QUAD12, KP_INT_EULER, false>(envs, n, lds, grid, s);
  return sym ? launch_prop_batch_t<KP_DYN_QUAD12, KP_INT_RK4, true>(envs, n, lds, grid, s)
              : launch_prop_batch_t<KP_DYN_QUAD12, KP_INT_RK4, false>(envs, n, lds, grid, s);
}

hipError_t launch_post_batch(const Env* const* envs, int n, int n_region, int n_commit,
                             int n_nodes, hipStream_t s) {
  if (n_commit < 1) n_commit = 1;
  if (n_nodes < 1) n_nodes = 1;
  hipLaunchKernelGGL(k_post_batch, dim3(n_region + n_commit + n_nodes, n), dim3(kCommitBlock), 0, s,
                     envs, n_commit);
  return hipGetLastError();
}

template <int DYN, int INTEG, bool SYM>
static hipError_t launch_queue_t(const Env* const* envs, const int32_t* order, const QueueJob* jobs,
                                 int n, QueueCtl* qc, unsigned long long* t_end, int32_t* ran,
                                 size_t lds, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_plan_queue<DYN, INTEG, SYM>), dim3(grid), dim3(kQueueBlock), (uint32_t)lds,
                     s, envs, order, jobs, n, qc, t_end, ran);
  return hipGetLastError();
}

hipError_t launch_plan_queue(int dyn, int integ, int sym, const Env* const* envs,
                             const int32_t* order, const QueueJob* jobs, int n, QueueCtl* qc,
                             unsigned long long* t_end, int32_t* ran, size_t lds, int grid,
                             hipStream_t s) {
  if (grid < 1) grid = 1;
  if (dyn == KP_DYN_DI6 && integ == KP_INT_EULER)
    return launch_queue_t<KP_DYN_DI6, KP_INT_EULER, false>(envs, order, jobs, n, qc, t_end, ran, lds,
                                                           grid, s);
  if (dyn == KP_DYN_DI6)
    return launch_queue_t<KP_DYN_DI6, KP_INT_RK4, false>(envs, order, jobs, n, qc, t_end, ran, lds,
                                                         grid, s);
  if (integ == KP_INT_EULER)
    return sym ? launch_queue_t<KP_DYN_QUAD12, KP_INT_EULER, true>(envs, order, jobs, n, qc, t_end,
                                                                   ran, lds, grid, s)
               : launch_queue_t<KP_DYN_QUAD12, KP_INT_EULER, false>(envs, order, jobs, n, qc, t_end,
                                                                    ran, lds, grid, s);
  return sym ? launch_queue_t<KP_DYN_QUAD12, KP_INT_RK4, true>(envs, order, jobs, n, qc, t_end, ran,
                                                               lds, grid, s)
             : launch_queue_t<KP_DYN_QUAD12, KP_INT_RK4, false>(envs, order, jobs, n, qc, t_end, ran,
                                                                lds, grid, s);
}

hipError_t launch_batch_status(const Env* const* envs, int n, BatchStatus* out, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_status, dim3((n + 255) / 256), dim3(256), 0, s, envs, n, out);
  return hipGetLastError();
}

hipError_t launch_set_done(const Env* env, int32_t code, hipStream_t s) {
  hipLaunchKernelGGL(k_set_done, dim3(1), dim3(64), 0, s, env, code);
  return hipGetLastError();
}

hipError_t launch_path_gather(const Env* env, int32_t len, float* out, hipStream_t s) {
  if (len < 1) return hipSuccess;
  hipLaunchKernelGGL(k_path_gather, dim3((len + 255) / 256), dim3(256), 0, s, env, len, out);
  return hipGetLastError();
}

hipError_t launch_path(const Env* env, int32_t node, hipStream_t s) {
  hipLaunchKernelGGL(k_path, dim3(1), dim3(64), 0, s, env, node);
  return hipGetLastError();
}

// Dynamic LDS above 64 KiB (obstacle tables of more than ~1500 boxes) needs
// each propagate kernel's limit raised once; gfx950 gives a workgroup up to
// 160 KiB.  Done before the first occupancy query (at problem creation), so
// never inside a captured graph.
template <int DYN, int INTEG, bool SYM>
static hipError_t allow_lds_t() {
  // the largest table: the double integrator's with the grid, the
  // quadcopter's with per-wave candidate lists
  const int bytes =
      (int)prop_lds_bytes(DYN, KP_MAX_OBSTACLES, DYN == KP_DYN_DI6 ? kGridMaxWords : 0);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_propagate<DYN, INTEG, SYM>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_propagate_batch<DYN, INTEG, SYM>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  const int qbytes = (int)prop_lds_bytes(DYN, KP_MAX_OBSTACLES,
                                         DYN == KP_DYN_DI6 ? kGridMaxWords : 0, kQueueBlock / 64);
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_plan_queue<DYN, INTEG, SYM>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, qbytes);
}
static hipError_t allow_lds_all() {
  static const hipError_t once = [] {
    hipError_t e = allow_lds_t<KP_DYN_DI6, KP_INT_EULER, false>();
    if (e == hipSuccess) e = allow_lds_t<KP_DYN_DI6, KP_INT_RK4, false>();
    if (e == hipSuccess) e = allow_lds_t<KP_DYN_QUAD12, KP_INT_EULER, false>();
    if (e == hipSuccess) e = allow_lds_t<KP_DYN_QUAD12, KP_INT_EULER, true>();
    if (e == hipSuccess) e = allow_lds_t<KP_DYN_QUAD12, KP_INT_RK4, false>();
    if (e == hipSuccess) e = allow_lds_t<KP_DYN_QUAD12, KP_INT_RK4, true>();
    return e;
  }();
  return once;
}

template <int DYN, int INTEG, bool SYM>
static int occ_prop_t(size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_propagate<DYN, INTEG, SYM>,
                                                    prop_block(DYN), lds) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

int occupancy_propagate(int dyn, int integ, int sym, size_t lds, int* blocks_per_cu) {
  int nb;
  // if raising the limit fails, launches above 64 KiB of LDS fail and
  // report it; clear the error so that it does not surface at another call
  if (allow_lds_all() != hipSuccess) (void)hipGetLastError();
  if (dyn == KP_DYN_DI6 && integ == KP_INT_EULER)
    nb = occ_prop_t<KP_DYN_DI6, KP_INT_EULER, false>(lds);
  else if (dyn == KP_DYN_DI6)
    nb = occ_prop_t<KP_DYN_DI6, KP_INT_RK4, false>(lds);
  else if (integ == KP_INT_EULER)
    nb = sym ? occ_prop_t<KP_DYN_QUAD12, KP_INT_EULER, true>(lds)
              : occ_prop_t<KP_DYN_QUAD12, KP_INT_EULER, false>(lds);
  else
    nb = sym ? occ_prop_t<KP_DYN_QUAD12, KP_INT_RK4, true>(lds)
              : occ_prop_t<KP_DYN_QUAD12, KP_INT_RK4, false>(lds);
  *blocks_per_cu = nb;
  return nb;
}

int occupancy_commit(int* blocks_per_cu) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_commit, kCommitBlock, 0) != hipSuccess)
    nb = 1;
  if (nb < 1) nb = 1;
  *blocks_per_cu = nb;
  return nb;
}

template <int DYN, int INTEG, bool SYM>
static int occ_queue_t(size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_plan_queue<DYN, INTEG, SYM>, kQueueBlock,
                                                    lds) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

int occupancy_queue(int dyn, int integ, int sym, size_t lds, int* blocks_per_cu) {
  int nb;
  if (allow_lds_all() != hipSuccess) (void)hipGetLastError();
  if (dyn == KP_DYN_DI6 && integ == KP_INT_EULER)
    nb = occ_queue_t<KP_DYN_DI6, KP_INT_EULER, false>(lds);
  else if (dyn == KP_DYN_DI6)
    nb = occ_queue_t<KP_DYN_DI6, KP_INT_RK4, false>(lds);
  else if (integ == KP_INT_EULER)
    nb = sym ? occ_queue_t<KP_DYN_QUAD12, KP_INT_EULER, true>(lds)
              : occ_queue_t<KP_DYN_QUAD12, KP_INT_EULER, false>(lds);
  else
    nb = sym ? occ_queue_t<KP_DYN_QUAD12, KP_INT_RK4, true>(lds)
              : occ_queue_t<KP_DYN_QUAD12, KP_INT_RK4, false>(lds);
  *blocks_per_cu = nb;
  return nb;
}

int occupancy_post(int* blocks_per_cu) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_post, kCommitBlock, 0) != hipSuccess)
    nb = 1;
  if (nb < 1) nb = 1;
  *blocks_per_cu = nb;
  return nb;
}

int occupancy_nodes(int* blocks_per_cu) {
  int a = 0, b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_nodesets, kNodeBlock, 0) != hipSuccess)
    a = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_frontier, kNodeBlock, 0) != hipSuccess)
    b = 1;
  int nb = a < b ? a : b;
  if (nb < 1) nb = 1;
  *blocks_per_cu = nb;
  return nb;
}

}  // namespace kp
