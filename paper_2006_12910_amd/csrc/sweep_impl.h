// sweep_impl.h -- the fused stream-collide sweep and the initial collision.
//
// One launch advances every tile of every domain of a batch by one step:
//   pull  f_i(x) <- f*_i(x - e_i) from the post-collision buffer of step T,
//         with halfway bounce-back where the source is solid, moving-wall
//         bounce-back where the pull crosses a particle surface (Eqs. MP7-MP8),
//         and Zou-He reconstruction of the unknown populations on density faces;
//   collide at step T+1: moments, body force through the equilibrium velocity
//         (Sec. 2), local power-law tau* (Sec. 5), BGK relaxation (Eq. LB1),
//         thermal noise on the non-conserved modes (Eqs. NP1-NP2);
//   store f*(T+1) into the other buffer.
// Arithmetic works on deviations d_i = f_i - w_i rho0 and never forms f_i.
#pragma once

#include <type_traits>

#include "lb_device.h"

namespace lbk {

template <class R> __device__ __forceinline__ R par(double a, float b);
template <> __device__ __forceinline__ double par<double>(double a, float) { return a; }
template <> __device__ __forceinline__ float par<float>(double, float b) { return b; }

template <class R> __device__ __forceinline__ R rsq(R v);
template <> __device__ __forceinline__ float rsq<float>(float v) { return 1.0f / sqrtf(v); }
template <> __device__ __forceinline__ double rsq<double>(double v) { return 1.0 / sqrt(v); }

template <class R> __device__ __forceinline__ R powr(R a, R b);
template <> __device__ __forceinline__ float powr<float>(float a, float b) { return exp2f(b * log2f(a)); }
template <> __device__ __forceinline__ double powr<double>(double a, double b) { return pow(a, b); }

// Local relaxation time of the power-law fluid (Sec. 5).  The shear rate
// comes from the non-equilibrium stress Pi = sum e e (f - feq(rho, j/rho + g/2)):
// gamma_dot = A / tau*, A = 3 |Pi|_F / (sqrt(2) rho).  With nu* = xi gamma_dot^(n-1)
// (Eq. nn4, kappa = 2^(n-1)) and tau* = 1/2 + 3 nu*, tau* is the root of
// h(tau) = tau - 1/2 - c tau^(1-n), c = 3 xi A^(n-1), clamped to
// [tau_min, tau_max].  n = 1/2 has the closed form tau = s^2,
// s = (c + sqrt(c^2 + 2))/2; otherwise Newton from the bracket end on the side
// where it converges monotonically (tau_max for n < 1, tau_min for n > 1).
template <class R, int PLM, int ST>
__device__ __forceinline__ R powerlaw_tau(const DevDomain &D, const R d[9], R drho, R rho, R irho,
                                          R jx, R jy) {
  const R gx = par<R>(D.gx, D.gx_f), gy = par<R>(D.gy, D.gy_f);
  const R ux = jx * irho + R(0.5) * gx, uy = jy * irho + R(0.5) * gy;
  const R third = drho * (R(1) / R(3));
  // d holds the stored scaling (see collide_node): axis values times K1,
  // diagonal values times K5, both powers of two
  constexpr R i1 = R(1) / R(kscale<ST>(1)), i5 = R(1) / R(kscale<ST>(5));
  const R dsum = (d[5] + d[6]) + (d[7] + d[8]);
  const R sxx = i1 * (d[1] + d[3]) + i5 * dsum;
  const R syy = i1 * (d[2] + d[4]) + i5 * dsum;
  const R sxy = i5 * ((d[5] - d[6]) + (d[7] - d[8]));
  const R pxx = sxx - rho * ux * ux - third;
  const R pyy = syy - rho * uy * uy - third;
  const R pxy = sxy - rho * ux * uy;
  const R fro = sqrt(pxx * pxx + pyy * pyy + R(2) * pxy * pxy);
  const R A = R(2.1213203435596424) * fro * irho;  // 3 / sqrt(2)
  const R tmin = par<R>(D.tau_min, D.tau_min_f), tmax = par<R>(D.tau_max, D.tau_max_f);
  const R xi = par<R>(D.pl_K, D.pl_K_f);
  const R n = par<R>(D.pl_n, D.pl_n_f);
  if (PLM == PL_GENERIC && n == R(1)) {  // Newtonian: tau* = 1/2 + 3 xi
    const R t = R(0.5) + R(3) * xi;
    return t < tmin ? tmin : (t > tmax ? tmax : t);
  }
  const bool thinning = PLM == PL_HALF || PLM == PL_3Q || (PLM == PL_GENERIC && n < R(1));
  if (!(A > R(0))) return thinning ? tmax : tmin;
  R tau;
  if constexpr (PLM == PL_HALF) {
    const R c = R(3) * xi * rsq<R>(A);
    const R s = R(0.5) * (c + sqrt(c * c + R(2)));
    tau = s * s;
  } else {
    R c;
    if constexpr (PLM == PL_3Q) c = R(3) * xi * sqrt(rsq<R>(A));          // A^(-1/4)
    else if constexpr (PLM == PL_3H) c = R(3) * xi * sqrt(A);              // A^(1/2)
    else c = R(3) * xi * powr<R>(A, n - R(1));
    // h(t) = t - 1/2 - c t^(1-n), h'(t) = 1 - c (1-n) t^(-n)
    auto tpow = [&](R t, R &tp, R &tpm) {  // t^(1-n), t^(-n)
      if constexpr (PLM == PL_3Q) { const R q = sqrt(sqrt(t)); tp = q; tpm = q / t; }
      else if constexpr (PLM == PL_3H) { const R r = rsq<R>(t); tp = r; tpm = r / t; }
      else { tp = powr<R>(t, R(1) - n); tpm = tp / t; }
    };
    R t0 = thinning ? tmax : tmin;
    R tp, tpm;
    tpow(t0, tp, tpm);
    const R h0 = t0 - R(0.5) - c * tp;
    if (thinning ? !(h0 > R(0)) : !(h0 < R(0))) return t0;
    constexpr int ITERS = sizeof(R) == 8 ? 40 : 12;
    const R tol = sizeof(R) == 8 ? R(1e-15) : R(1e-7);
    R t = t0;
#pragma unroll 1
    for (int it = 0; it < ITERS; ++it) {
      tpow(t, tp, tpm);
      const R h = t - R(0.5) - c * tp;
      const R dh = R(1) - c * (R(1) - n) * tpm;
      const R tn = t - h / dh;
      const bool done = fabs(tn - t) <= tol * tn;
      t = tn;
      if (done) break;
    }
    tau = t;
  }
  return tau < tmin ? tmin : (tau > tmax ? tmax : tau);
}

// Reciprocal of the density: FP32 takes the hardware estimate (1 ulp) and,
// for FP32 storage, one Newton step (error below one ulp); with 16-bit
// storage the estimate alone, whose error is four orders below the stored
// values' spacing.  FP64: the correctly rounded division.  The reciprocal
// enters only the second-order term of the equilibrium (the momentum part
// is built from J itself), so it does not touch mass or momentum.
template <int ST, class R> __device__ __forceinline__ R recip(R x) {
  if constexpr (sizeof(R) == 8) {
    return R(1) / x;
  } else {
    const float r = __builtin_amdgcn_rcpf(x);
    if constexpr (ST == ST_F16 || ST == ST_BF16) return r;
    else return fmaf(fmaf(-x, r, 1.0f), r, r);
  }
}

// Fused multiply-add in the arithmetic type.  The library is compiled without
// floating-point contraction (so every kernel rounds a node's arithmetic the
// same way); the products that should fuse are written with fmar.
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// delta rho of deviations in the stored scaling (the factors are powers of
// two, so the fused form rounds as the sum of the scaled values)
template <int ST, class R> __device__ __forceinline__ R scaled_drho(const R d[9]) {
  constexpr R i0 = R(1) / R(kscale<ST>(0)), i1 = R(1) / R(kscale<ST>(1)), i5 = R(1) / R(kscale<ST>(5));
  // the diagonal pairs (5, 6) and (7, 8) are the ones the y momentum sums
  return fmar(i0, d[0], fmar(i1, (d[1] + d[3]) + (d[2] + d[4]), i5 * ((d[5] + d[6]) + (d[7] + d[8]))));
}

// a + b in FP32 rounded stochastically: the exact sum s + e (s = fl(a + b),
// e from Knuth's TwoSum, exact without contraction) lies between s and its
// neighbour one ulp toward e; the neighbour is taken when |e| exceeds a
// uniform fraction (the top 24 bits of r) of the distance to it, i.e. with
// probability |e| / ulp.
__device__ __forceinline__ float sr_add_f32(float a, float b, uint32_t r) {
#pragma clang fp contract(off)
  const float s = a + b;
  const float bb = s - a;
  const float e = (a - (s - bb)) + (b - bb);
  const uint32_t us = __float_as_uint(s);
  // magnitude one step up where e has the sign of s, else one step down (s is
  // never zero when e is not)
  const uint32_t un = ((__float_as_uint(e) ^ us) & 0x80000000u) ? us - 1u : us + 1u;
  const float t = __uint_as_float(un) - s;
  const float u = (float)(r >> 8) * 5.9604644775390625e-8f;  // 2^-24
  return (e != 0.0f && fabsf(e) > u * fabsf(t)) ? __uint_as_float(un) : s;
}

// BGK (or, with F_TRT, two-relaxation-time) collision of one node, step
// `step`, in arithmetic type R.  The values
// are the deviations d_i = f_i - w_i rho0 in the stored scaling: times K0, K1,
// K5 for rest, axis and diagonal directions (powers of two: 2, 8, 32 for the
// 16-bit formats, 1 otherwise).  Scaling by a power of two commutes with every
// rounding, so the result is exactly K_i times the unscaled computation, and
// the stores and loads need no conversion factor.
//
// The equilibrium of Eq. LB2 with u = j/rho + tau g is evaluated in a form
// whose mass and momentum do not depend on how the lattice constants round:
// the linear term is built from J = j + rho tau g with coefficients L1 ~ 1/3,
// L5 = (1 - 2 L1)/4 (so 2 L1 + 4 L5 = 1 exactly), opposite directions share
// one even part c and take c +- (linear term), and the rest population is
// delta_rho minus the other eight.  Algebraically this is Eq. LB2; in FP32 it
// removes a systematic O(1e-8) momentum error per step that would otherwise
// bias slowly accelerating flows.
template <int ST, int FEAT, int PLM, class R>
__device__ __forceinline__ void collide_node(const DevDomain &D, R d[9], uint32_t node,
                                             uint32_t step) {
  constexpr R K0 = R(kscale<ST>(0)), K1 = R(kscale<ST>(1)), K5 = R(kscale<ST>(5));
  constexpr R i1 = R(1) / K1, i5 = R(1) / K5;
  const R drho = scaled_drho<ST, R>(d);
  const R jx = fmar(i1, d[1] - d[3], i5 * ((d[5] - d[6]) + (d[8] - d[7])));
  const R jy = fmar(i1, d[2] - d[4], i5 * ((d[5] + d[6]) - (d[7] + d[8])));
  const R rho = par<R>(D.rho0, D.rho0_f) + drho;
  const R irho = recip<ST, R>(rho);
  constexpr bool TRT = (FEAT & F_TRT) != 0;
  R tau, om;
  if constexpr ((FEAT & F_POWER) != 0) {
    tau = powerlaw_tau<R, PLM, ST>(D, d, drho, rho, irho, jx, jy);
    om = R(1) / tau;
  } else {
    tau = par<R>(D.tau, D.tau_f);
    om = par<R>(D.omega, D.omega_f);
  }
  // TRT: the antisymmetric parts relax with 1/tau_m and carry the momentum,
  // so the force shifts u_eq by tau_m g (BGK: tau_m = tau)
  R taum = tau, omm = om;
  if constexpr (TRT) {
    if constexpr ((FEAT & F_POWER) != 0) {
      taum = R(0.5) + par<R>(D.magic, D.magic_f) / (tau - R(0.5));
      omm = R(1) / taum;
    } else {
      taum = par<R>(D.tau_m, D.tau_m_f);
      omm = par<R>(D.omega_m, D.omega_m_f);
    }
  }
  const R rt = rho * taum;
  const R Jx = fmar(rt, par<R>(D.gx, D.gx_f), jx);
  const R Jy = fmar(rt, par<R>(D.gy, D.gy_f), jy);
  const R ux = Jx * irho, uy = Jy * irho;
  const R W1 = R(1) / R(9), W5 = R(0.25) * W1;
  const R L1 = R(1) / R(3), L5 = (R(1) - R(2) * L1) * R(0.25);
  const R q = (R(1.5) * rho) * fmar(ux, ux, uy * uy);
  const R sp = ux + uy, sm = uy - ux;
  // even parts and linear terms of omega feq, already in the stored scaling:
  // omega rides on the class coefficients (uniform unless the relaxation
  // time is local), so the relaxation below is one fused multiply-add a
  // direction, d (1 - omega) + omega feq, instead of a subtraction and one
  R aw1, aw5, al1, al5, aq1, aq5;
  if constexpr (TRT) {  // feq itself: the two rates act in the relaxation
    aw1 = K1 * W1;
    aw5 = K5 * W5;
    al1 = K1 * L1;
    al5 = K5 * L5;
    aq1 = R(4.5) * aw1;
    aq5 = R(4.5) * aw5;
  } else if constexpr ((FEAT & F_POWER) != 0) {
    aw1 = om * (K1 * W1);
    aw5 = om * (K5 * W5);
    al1 = om * (K1 * L1);
    al5 = om * (K5 * L5);
    aq1 = R(4.5) * aw1;
    aq5 = R(4.5) * aw5;
  } else {  // the same products, formed once on the host
    aw1 = par<R>(D.cw1, D.cw1_f);
    aw5 = par<R>(D.cw5, D.cw5_f);
    al1 = par<R>(D.cl1, D.cl1_f);
    al5 = par<R>(D.cl5, D.cl5_f);
    aq1 = par<R>(D.cq1, D.cq1_f);
    aq5 = par<R>(D.cq5, D.cq5_f);
  }
  // even part of class k: aw_k (drho - q) + aw_k (9/2) rho (e.u)^2
  const R t0 = drho - q;
  const R b1 = aw1 * t0, b5 = aw5 * t0;
  const R a1 = aq1 * rho, a5 = aq5 * rho;
  const R cxx = fmar(a1 * ux, ux, b1);
  const R cyy = fmar(a1 * uy, uy, b1);
  const R cpp = fmar(a5 * sp, sp, b5);
  const R cmm = fmar(a5 * sm, sm, b5);
  const R lx = al1 * Jx, ly = al1 * Jy;
  const R lp = al5 * (Jx + Jy), lm = al5 * (Jy - Jx);
  R eq[9];  // omega feq_i (BGK), feq_i (TRT)
  eq[0] = K0 * fmar(R(-2), fmar(i1, cxx + cyy, i5 * (cpp + cmm)), TRT ? drho : om * drho);
  // TRT relaxation of the pair (i, o = opposite): the symmetric part of
  // feq - d with omega, the antisymmetric part with omega_m
  auto trt_pair = [&](int i, int o, R &di, R &dout) {
    const R a = eq[i] - d[i], b = eq[o] - d[o];
    const R sym = R(0.5) * (a + b), anti = R(0.5) * (a - b);
    const R t = omm * anti;
    di = fmar(om, sym, t);
    dout = fmar(om, sym, -t);
  };
  eq[1] = cxx + lx;
  eq[3] = cxx - lx;
  eq[2] = cyy + ly;
  eq[4] = cyy - ly;
  eq[5] = cpp + lp;
  eq[7] = cpp - lp;
  eq[6] = cmm + lm;
  eq[8] = cmm - lm;

  // thermal noise zeta_i of Eqs. NP1-NP2 (zero mass and momentum):
  // zeta_i = amp w_i z_i, z_i = sum_k e_ki t_k over the Table t1 basis
  // polynomials of the six non-conserved modes, t_k = Theta_k / sqrt(w_k).
  // Opposite directions share the even part of z and take +- the odd part;
  // add(i, c, z) receives the coefficient amp w_i (stored scaling) and z_i.
  auto noise = [&](auto &&add) {
    float th[6];
    noise_normals<sizeof(R) == 4>(D.key0, D.key1, node, step, th);
    // Theta_k / sqrt(w_k) with w_k = 4, 4/9, 1/9, 2/3, 2/3, 16 (Table t1)
    const R t3 = R(th[0]) * R(0.5), t4 = R(th[1]) * R(1.5), t5 = R(th[2]) * R(3);
    const R t6 = R(th[3]) * R(1.2247448713915890491), t7 = R(th[4]) * R(1.2247448713915890491);
    const R t8 = R(th[5]) * R(0.25);
    const R amp = sqrt(rho * par<R>(D.kT, D.kT_f) * om * (R(2) - om) * R(3));
    // e_k of rest: (-2, 0, 0, 0, 0, 2); axis (1, 0): (1, 1, 0, -1, 0, -4);
    // diagonal (1, 1): (4, 0, 1, 2, 2, 8), the others by symmetry
    const R a0 = fmar(R(-4), t8, t3);      // t3 - 4 t8
    const R ax = a0 + t4, ay = a0 - t4;     // even parts, x and y axis
    const R d0 = fmar(R(4), t3, R(8) * t8);  // 4 t3 + 8 t8
    const R dp = d0 + t5, dm = d0 - t5;     // even parts, diagonals 5/7 and 6/8
    const R op = R(2) * (t6 + t7), om2 = R(2) * (t7 - t6);
    const R c0 = amp * (K0 * (R(4) * W1)), c1 = amp * (K1 * W1), c5 = amp * (K5 * W5);
    add(0, c0, R(2) * (t8 - t3));
    add(1, c1, ax - t6);
    add(3, c1, ax + t6);
    add(2, c1, ay - t7);
    add(4, c1, ay + t7);
    add(5, c5, dp + op);
    add(7, c5, dp - op);
    add(6, c5, dm + om2);
    add(8, c5, dm - om2);
  };

  if constexpr (ST == ST_F32 && sizeof(R) == 4) {
    // FP32 storage with FP32 arithmetic: the step is formed as an increment
    // inc_i = omega (feq_i - d_i) (+ zeta_i) whose mass and momentum are
    // then made exactly those of the method (zero and rho g: the collision
    // conserves mass and adds the body force, Sec. 2) from sums of the small
    // increments, and d_i + inc_i is rounded once.  The populations carry
    // the momentum term 3 w rho e.u (~1e-2 at u = 0.05), whose FP32 spacing
    // (~2e-9) is comparable to a step's momentum input rho g in slow forced
    // flows (2e-8 in the n = 1.5 power-law channel): rounded in the
    // relaxation, the momentum change was biased by up to ~20 % of rho g at
    // each node, steadily, and the channel drifted 4e-5 from the FP64
    // result within 1500 steps.  With the correction the FP32 arithmetic
    // adds no bias beyond the storage rounding itself.  The rest population
    // takes the mass balance, so its equilibrium value is not needed.
    R inc[9];
    if constexpr (TRT) {
      trt_pair(1, 3, inc[1], inc[3]);
      trt_pair(2, 4, inc[2], inc[4]);
      trt_pair(5, 7, inc[5], inc[7]);
      trt_pair(6, 8, inc[6], inc[8]);
    } else {
#pragma unroll
      for (int i = 1; i < 9; ++i) inc[i] = fmar(-om, d[i], eq[i]);
    }
    if constexpr ((FEAT & F_NOISE) != 0)
      noise([&](int i, R c, R z) { if (i > 0) inc[i] = fmar(c, z, inc[i]); });
    const R sx = ((inc[1] - inc[3]) + (inc[5] - inc[6])) + (inc[8] - inc[7]);
    const R sy = ((inc[2] - inc[4]) + (inc[5] + inc[6])) - (inc[7] + inc[8]);
    const R hx = R(0.5) * fmar(rho, par<R>(D.gx, D.gx_f), -sx);
    const R hy = R(0.5) * fmar(rho, par<R>(D.gy, D.gy_f), -sy);
    inc[1] += hx;
    inc[3] -= hx;
    inc[2] += hy;
    inc[4] -= hy;
    inc[0] = -(((inc[1] + inc[3]) + (inc[2] + inc[4])) + ((inc[5] + inc[7]) + (inc[6] + inc[8])));
    if (D.feat & F_STOCH) {
      // stochastic rounding of d_i + inc_i (uniform per domain): unbiased,
      // so increments smaller than half the spacing of the stored values
      // still move the state on average
      const uint32_t h = mix32(node ^ (mix32(step ^ D.key0) ^ D.key1));
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int r = (7 * i) & 31;
        d[i] = sr_add_f32(d[i], inc[i], r == 0 ? h : (h << r) | (h >> (32 - r)));
      }
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) d[i] = d[i] + inc[i];
    }
  } else if constexpr (TRT) {
    R u[9];
    u[0] = om * (eq[0] - d[0]);
    trt_pair(1, 3, u[1], u[3]);
    trt_pair(2, 4, u[2], u[4]);
    trt_pair(5, 7, u[5], u[7]);
    trt_pair(6, 8, u[6], u[8]);
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = d[i] + u[i];
  } else {
    const R keep = R(1) - om;
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = fmar(keep, d[i], eq[i]);
    if constexpr ((FEAT & F_NOISE) != 0) noise([&](int i, R c, R z) { d[i] = fmar(c, z, d[i]); });
  }
}

// Stored form of the nine post-collision deviations of one node.  16-bit
// storage with stochastic rounding takes its rounding bits from one hash of
// (node, step, key) per node, rotated by 7 i bits for direction i (nine
// distinct rotations), so every store of the same value at the same node and
// step rounds the same way.
template <int ST, class R, bool SR>
__device__ __forceinline__ void encode_node(const DevDomain &D, const R d[9], uint32_t node,
                                            uint32_t step, typename Store<ST>::T q[9]) {
  using S = Store<ST>;
  using RS = typename S::R;
  if constexpr (SR && (ST == ST_F16 || ST == ST_BF16)) {
    const uint32_t h = mix32(node ^ (mix32(step ^ D.key0) ^ D.key1));
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int r = (7 * i) & 31;
      q[i] = S::raw_sr((RS)d[i], r == 0 ? h : (h << r) | (h >> (32 - r)));
    }
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) q[i] = S::raw_rn((RS)d[i]);
  }
}


template <int ST, class R>
__device__ __forceinline__ void store_node(const DevDomain &D, typename Store<ST>::T *dst,
                                           size_t plane, uint32_t off, const R d[9],
                                           uint32_t node, uint32_t step) {
  typename Store<ST>::T q[9];
  if ((ST == ST_F16 || ST == ST_BF16) && (D.feat & F_STOCH)) encode_node<ST, R, true>(D, d, node, step, q);
  else encode_node<ST, R, false>(D, d, node, step, q);
#pragma unroll
  for (int i = 0; i < 9; ++i) gbl(dst + i * plane)[off] = q[i];
}

// Arithmetic type: FP64 for FP64 storage or when wide arithmetic is chosen,
// FP32 otherwise.
template <int ST, int WIDE>
using CompT = typename std::conditional<ST == ST_F64 || WIDE != 0, double, float>::type;

// Rows a thread loads before it computes: 16-bit storage moves half the bytes
// per load, so it keeps more rows in flight to cover memory latency.
template <int ST> constexpr int rows_in_flight() { return ST == ST_F16 || ST == ST_BF16 ? 4 : 2; }

// The sweep addresses a population buffer through a raw buffer resource
// (base, size in bytes; a domain's nine planes span fewer than 2^32 bytes).
// A buffer access adds a scalar and a vector byte offset in the memory unit:
// the plane and row part of every offset is wave-uniform (scalar adds) and
// the vector part is the column, so the pulls and stores of a node need no
// vector address arithmetic.  Word 3 is the raw-buffer format of the gfx9
// family.
typedef __amdgpu_buffer_rsrc_t BufRes;
__device__ __forceinline__ BufRes pop_buffer(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
template <class T> __device__ __forceinline__ T bload(BufRes r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 2) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0));
  } else if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
  } else {
    static_assert(sizeof(T) == 8, "population type");
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
  }
}
// NT: non-temporal store.  A written line is read again only in the next
// step; once a step's working set exceeds the caches it would be evicted
// before then, so caching it only displaces the source rows still being
// pulled.
template <class T, bool NT>
__device__ __forceinline__ void bstore(BufRes r, uint32_t voff, uint32_t soff, T v) {
  constexpr int aux = NT ? 2 : 0;  // cache-policy bits: 2 = nt
  if constexpr (sizeof(T) == 2) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, (int)voff, (int)soff, aux);
  } else if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, aux);
  } else {
    static_assert(sizeof(T) == 8, "population type");
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, aux);
  }
}

// Pull of one node.  Every direction loads the neighbour's slot at x - e_i,
// except where that neighbour is a stationary solid node of the label plane
// (bit i-1 of `solid_src`): then halfway bounce-back loads this node's own
// slot of the opposite direction.  Index walls of a label-free domain have
// their slots filled by mirror writes instead (see k_sweep), and where the
// pull crosses a particle surface the neighbour's slot already holds the
// moving-wall bounced value, put there by the particle pre-pass (k_pre).  A
// source beyond a density face is read from the node's own column: those
// populations are unknown and the face reconstruction replaces them.  row[]
// (wave-uniform) and col[] are the byte offsets of the (wrapped or clamped)
// source rows y+1, y, y-1 and columns x+1, x, x-1.  With labels, the scalar
// offset of direction i is the smaller of the two candidates' uniform parts
// (opposite directions lie two planes apart, so which one is smaller is
// known at compile time) and the vector offset adds the difference, which is
// never negative.
template <class T, bool LABELS, class P>
__device__ __forceinline__ void pull_node(BufRes src, uint32_t planeB, const uint32_t (&row)[3],
                                          const uint32_t (&col)[3], uint32_t solid_src, P &raw) {
  raw.set(0, bload<T>(src, col[1], row[1]));
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const uint32_t sN = (uint32_t)i * planeB + row[1 + cy(i)];  // neighbour's slot
    const uint32_t vN = col[1 + cx(i)];
    if constexpr (!LABELS) {
      raw.set(i, bload<T>(src, vN, sN));
    } else {
      const uint32_t sB = (uint32_t)opp(i) * planeB + row[1];  // own opposite slot
      // all ones where the pull bounces back, else zero; a ^ ((a ^ b) & m)
      // picks b under the mask (one three-input bitwise instruction)
      // (the empty asm operands keep the optimiser from turning the mux back
      // into a compare and select, and from splitting the scalar delta)
      uint32_t m = (uint32_t)(-(int32_t)((solid_src >> (i - 1)) & 1u));
      __asm__("" : "+v"(m));
      if (opp(i) > i) {  // resolved at compile time once the loop is unrolled
        uint32_t d = sB - sN;
        __asm__("" : "+s"(d));
        const uint32_t vB = col[1] + d;
        raw.set(i, bload<T>(src, vN ^ ((vN ^ vB) & m), sN));
      } else {
        uint32_t d = sN - sB;
        __asm__("" : "+s"(d));
        const uint32_t vA = vN + d;
        raw.set(i, bload<T>(src, vA ^ ((vA ^ col[1]) & m), sB));
      }
    }
  }
}

// Stored values of one node while its loads are in flight (decoded only
// when the node is computed).
template <class T> struct Pulled {
  T v[9];
  __device__ __forceinline__ void set(int i, T x) { v[i] = x; }
  __device__ __forceinline__ T get(int i) const { return v[i]; }
};
// 16-bit values two to a register (loads into the low and high halves), which
// halves the registers that hold the rows in flight
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
template <> struct Pulled<uint16_t> {
  u16x2 v[5];
  __device__ __forceinline__ void set(int i, uint16_t x) { v[i >> 1][i & 1] = x; }
  __device__ __forceinline__ uint16_t get(int i) const { return v[i >> 1][i & 1]; }
};

// Byte offsets of the source rows y+1, y, y-1 (index 1 + cy): wrapped on a
// periodic axis, else a row beyond the edge is clamped to y.
__device__ __forceinline__ void src_rows(int y, int ny, uint32_t pitchB, uint32_t planeB,
                                         bool periodic, uint32_t (&row)[3]) {
  const uint32_t yp = (uint32_t)y * pitchB;
  row[1] = yp;
  row[0] = y + 1 < ny ? yp + pitchB : (periodic ? 0u : yp);
  row[2] = y > 0 ? yp - pitchB : (periodic ? planeB - pitchB : yp);
}

// Bit i-1 set for the directions i with cx(i) == v (resp. cy(i) == v).
constexpr uint32_t dirs_cx(int v) {
  uint32_t m = 0;
  for (int i = 1; i < 9; ++i) m |= cx(i) == v ? 1u << (i - 1) : 0u;
  return m;
}
constexpr uint32_t dirs_cy(int v) {
  uint32_t m = 0;
  for (int i = 1; i < 9; ++i) m |= cy(i) == v ? 1u << (i - 1) : 0u;
  return m;
}

// 256 threads.  The plain and obstacle variants are held to at least 5 waves
// per SIMD (enough loads in flight to cover memory latency, no spills); the
// noise and power-law variants keep the compiler's register choice.
template <int FEAT, int WIDE> constexpr int sweep_min_waves() {
  return (FEAT & (F_NOISE | F_POWER)) == 0 && WIDE == 0 ? 5 : 1;
}

template <int ST, int FEAT, int PLM, int WIDE>
__global__ __launch_bounds__(256, (sweep_min_waves<FEAT, WIDE>())) void k_sweep(
    const DevDomain *__restrict__ doms, const int *__restrict__ prefix, int ndom, int kstep,
    int part) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = CompT<ST, WIDE>;
  constexpr bool LABELS = (FEAT & F_LABELS) != 0;
  constexpr int U = rows_in_flight<ST>();
  constexpr uint32_t B = sizeof(T);

  const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int dix = ndom == 1 ? 0 : find_domain(prefix, ndom, b);
  const DevDomain &D = doms[dix];
  const int local = b - prefix[dix];
  const int nx = D.nx, ny = D.ny, pitch = D.pitch;
  const int tw = D.tile_w, npt = D.rows_per_thread;
  const int rows_pass = 256 / tw;
  const int tyi = local / D.tiles_x, txi = local - tyi * D.tiles_x;
  const int x = txi * tw + (int)threadIdx.x % tw;
  if (x >= nx) return;
  // tile widths are multiples of 64, so all lanes of a wave share one row:
  // the row index and everything derived from it (validity, wrapped
  // neighbour rows, row offsets) is wave-uniform and lives in scalar registers
  const int ybase = __builtin_amdgcn_readfirstlane(tyi * rows_pass * npt + (int)threadIdx.x / tw);

  const uint64_t T0 = *gbl(D.tstep) + (uint64_t)kstep;  // state time of the source buffer
  // part 1: only the tiles that no particle coupling of this step touches;
  // part 2: only those it touches (the two launches of an overlapped step);
  // 0: every tile.  Uniform over the workgroup, and k_sweep has no barrier.
  if (part != 0) {
    const bool near = gbl(D.near_tiles[T0 & 1])[local] != 0;
    if (near != (part == 2)) return;
  }
  const uint32_t step = (uint32_t)(T0 + 1);
  void *const f0 = D.f[0];
  void *const f1 = D.f[1];
  const uint32_t nbytes = 9u * (uint32_t)ny * (uint32_t)pitch * (uint32_t)sizeof(T);
  const BufRes src = pop_buffer((T0 & 1) ? f1 : f0, nbytes);
  const BufRes dst = pop_buffer((T0 & 1) ? f0 : f1, nbytes);
  const uint32_t pitchB = (uint32_t)pitch * B;
  const uint32_t planeB = (uint32_t)ny * pitchB;
  bool bad = false;  // non-finite density seen by this thread
  const bool perx = D.bc_x == BC_PERIODIC, wallx = D.bc_x == BC_WALL;
  const bool pery = D.bc_y == BC_PERIODIC, wally = D.bc_y == BC_WALL;
  const bool pressx = D.bc_x == BC_PRESSURE;
  // a batch may mix domains with and without a label plane
  const bool has_lab = LABELS && D.label != nullptr;
  // index walls of a domain without a label plane
  const bool walls = !has_lab && (wallx || wally);
  // nodes on a density face (Zou-He reconstruction)
  const bool face = pressx && (x == 0 || x == nx - 1);

  // source columns x+1, x, x-1 (index 1 + cx); a column beyond a
  // non-periodic edge is clamped to x
  uint32_t colv[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int c = x + 1 - k;
    colv[k] = (uint32_t)(c < 0 ? (perx ? c + nx : x) : (c >= nx ? (perx ? c - nx : x) : c)) * B;
  }
  // index walls: directions whose source is a wall column, and directions
  // whose source column lies inside the domain
  const uint32_t wall_cols =
      wallx ? (x == 1 ? dirs_cx(1) : 0u) | (x == nx - 2 ? dirs_cx(-1) : 0u) : 0u;
  const uint32_t cols_in = 0xffu & ~(!perx && x == 0 ? dirs_cx(1) : 0u) &
                           ~(!perx && x == nx - 1 ? dirs_cx(-1) : 0u);

  // node words of a row group; a clamped row's word must not act.  Every pull
  // address of a labelled node depends on its word, so the words of the next
  // group are loaded while the current group's pulls are in flight.
  auto load_words = [&](int r0, uint32_t (&w)[U]) {
    int yg = ybase + r0 * rows_pass;
    __asm__ volatile("" : "+s"(yg));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int yr = yg + u * rows_pass;
      const bool valid = r0 + u < npt && yr < ny;
      const int y = valid ? yr : ny - 1;
      const uint32_t v = gbl(D.nodew)[(uint32_t)y * pitch + x];
      w[u] = valid ? v : 0u;
    }
  };
  uint32_t nwn[U];
#pragma unroll
  for (int u = 0; u < U; ++u) nwn[u] = 0;
  if (has_lab) load_words(0, nwn);

#pragma unroll 1
  for (int r0 = 0; r0 < npt; r0 += U) {
    uint32_t nw[U];
#pragma unroll
    for (int u = 0; u < U; ++u) nw[u] = nwn[u];
    if (has_lab && r0 + U < npt) load_words(r0 + U, nwn);
    // first row of this group and the column offsets, hidden from the
    // optimiser so that it neither turns every address of the group into an
    // induction variable of its own nor keeps a loop-invariant partial sum
    // per direction in a register
    int yg = ybase + r0 * rows_pass;
    uint32_t col[3] = {colv[0], colv[1], colv[2]};
    __asm__ volatile("" : "+s"(yg), "+v"(col[0]), "+v"(col[1]), "+v"(col[2]));
    Pulled<T> raw[U];
    bool act[U];
    // phase 1: every load of the row group, branch-free and none depending on
    // another, so they are all in flight together; rows past the tile or the
    // domain load from a clamped valid row and are discarded
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int yr = yg + u * rows_pass;
      const bool valid = r0 + u < npt && yr < ny;
      const int y = valid ? yr : ny - 1;
      const bool wall =
          walls && ((wally && (y == 0 || y == ny - 1)) || (wallx && (x == 0 || x == nx - 1)));
      act[u] = valid && !wall;
      uint32_t row[3];
      src_rows(y, ny, pitchB, planeB, pery, row);
      pull_node<T, LABELS>(src, planeB, row, col, nw[u] & 0xffu, raw[u]);
    }
    // phase 2: boundary reconstruction, collision, stores
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int y = yg + u * rows_pass;
      if (!act[u]) continue;
      // a stationary solid node of the label plane is swept as a node at rest
      // (zero deviations): its slots are never pulled (the pulls next to it
      // bounce back on their own slots), but storing them keeps every slot of
      // the buffer written once a step, with no cache line written in part
      // (a partial line costs the memory a read-modify-write), and keeps the
      // lanes of a wave on one path
      const bool solid = LABELS && (nw[u] & NODE_SOLID);
      R e[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) e[i] = solid ? R(0) : (R)S::raw_dec(raw[u].get(i));
      if (face) {
        // 2/3 + 2 (1/6) = 1 exactly in the chosen constants; unscaled values
        const R half = R(0.5), third2 = R(2) / R(3), sixth = (R(1) - third2) * R(0.5);
#pragma unroll
        for (int i = 0; i < 9; ++i) e[i] *= R(1) / R(kscale<ST>(i));
        if (x == 0) {
          const R s = e[0] + e[2] + e[4] + R(2) * (e[3] + e[6] + e[7]);
          const R rux = par<R>(D.drho_in, D.drho_in_f) - s;
          e[1] = e[3] + third2 * rux;
          e[5] = e[7] - half * (e[2] - e[4]) + sixth * rux;
          e[8] = e[6] + half * (e[2] - e[4]) + sixth * rux;
        } else {
          const R s = e[0] + e[2] + e[4] + R(2) * (e[1] + e[5] + e[8]);
          const R rux = s - par<R>(D.drho_out, D.drho_out_f);
          e[3] = e[1] - third2 * rux;
          e[7] = e[5] + half * (e[2] - e[4]) - sixth * rux;
          e[6] = e[8] - half * (e[2] - e[4]) - sixth * rux;
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) e[i] *= R(kscale<ST>(i));
      }
      const uint32_t node = (uint32_t)y * (uint32_t)nx + (uint32_t)x;
      // non-finite check on the pulled density (the collision computes the
      // same sum): a blow-up is seen one step after it is stored, and the
      // density reduction after every call covers the final state
      bad = bad || !(fabs(scaled_drho<ST, R>(e)) < R(1e30));
      collide_node<ST, FEAT, PLM, R>(D, e, node, step);
      uint32_t row[3];  // rows y + 1, y, y - 1; all inside the domain for a computed node
      src_rows(y, ny, pitchB, planeB, true, row);
      // index walls of a label-free domain: mirror writes (bit i-1: the
      // source x - e_i is a wall node)
      uint32_t mb = 0;
      if (walls) {
        const uint32_t wall_rows =
            wally ? (y == 1 ? dirs_cy(1) : 0u) | (y == ny - 2 ? dirs_cy(-1) : 0u) : 0u;
        mb = (wall_cols | wall_rows) & cols_in;
      }
      // the rounding mode is uniform: each branch keeps its stores, so neither
      // conversion is evaluated for the other
      auto emit = [&](auto sr_tag) {
        T q[9];
        encode_node<ST, R, decltype(sr_tag)::value>(D, e, node, step, q);
        // cache-resident working sets keep ordinary stores (the next step
        // reads them back from the cache); larger ones stream (stb_nt)
        if (D.stream_stores) {
#pragma unroll
          for (int i = 0; i < 9; ++i) bstore<T, true>(dst, col[1], (uint32_t)i * planeB + row[1], q[i]);
        } else {
#pragma unroll
          for (int i = 0; i < 9; ++i) bstore<T, false>(dst, col[1], (uint32_t)i * planeB + row[1], q[i]);
        }
        // mirror writes: the pull along i from the wall node x - e_i will
        // read this node's post-collision opposite population there, stored
        // exactly as the node's own slot of that direction
        if (mb) {
#pragma unroll
          for (int i = 1; i < 9; ++i) {
            if (!((mb >> (i - 1)) & 1u)) continue;
            bstore<T, false>(dst, col[1 + cx(i)], (uint32_t)i * planeB + row[1 + cy(i)], q[opp(i)]);
          }
        }
      };
      if ((ST == ST_F16 || ST == ST_BF16) && (D.feat & F_STOCH)) emit(std::true_type{});
      else emit(std::false_type{});
    }
  }
  if (bad) atomicOr(D.health, HEALTH_NONFINITE);
}

// Initial state: equilibrium of the given fields (or rest), then the
// collision of the current step, written to the buffer of that step.
// Rows [row0, row0 + nrows); fields are band-local [nrows][nx] FP64.
template <int ST, int FEAT, int PLM, int WIDE>
__global__ __launch_bounds__(256) void k_init(const DevDomain *__restrict__ Dp, const double *rho_f,
                                              const double *ux_f, const double *uy_f, int row0,
                                              int nrows) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = CompT<ST, WIDE>;
  const DevDomain &D = *Dp;
  const int x = (int)(blockIdx.x * 256 + threadIdx.x) % D.pitch;
  const int yl = (int)(blockIdx.x * 256 + threadIdx.x) / D.pitch;
  if (x >= D.nx || yl >= nrows) return;
  const int y = row0 + yl;
  const uint64_t T0 = *D.tstep;
  T *dst = (T *)D.f[T0 & 1];
  const size_t plane = (size_t)D.ny * D.pitch;
  const uint32_t here = (uint32_t)y * D.pitch + x;
  R d[9];
  if (rho_f) {
    const size_t fi = (size_t)yl * D.nx + x;
    const R rho = R(rho_f[fi]), ux = R(ux_f[fi]), uy = R(uy_f[fi]);
    const R drho = R(rho_f[fi] - D.rho0);
    const R A = drho - R(1.5) * rho * (ux * ux + uy * uy);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const R eu = R(3) * (R(cx(i)) * ux + R(cy(i)) * uy);
      d[i] = R(kscale<ST>(i)) * (wgt<R>(i) * (A + rho * (eu + R(0.5) * eu * eu)));
    }
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = R(0);
  }
  const uint32_t node = (uint32_t)y * (uint32_t)D.nx + (uint32_t)x;
  collide_node<ST, FEAT, PLM, R>(D, d, node, (uint32_t)T0);
  store_node<ST, R>(D, dst, plane, here, d, node, (uint32_t)T0);
}

}  // namespace lbk
