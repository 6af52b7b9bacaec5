// sweep3_impl.h -- the D3Q19 and D3Q27 variants of the fused stream-collide
// sweep (the three-dimensional lattices the paper names as its next step,
// Sec. 8): BGK
// or two-relaxation-time collision with the velocity-shift body force of
// Sec. 2, pull streaming with periodic wrap and halfway bounce-back on solid
// nodes, FP64, FP32, FP16 or BF16 storage of the deviations
// d_i = f_i - w_i rho0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lb_device.h"  // 16-bit conversions and the rounding-bit hash

namespace lbk3 {

// Rest, six axis velocities, twelve edge velocities (D3Q19), then eight
// corner velocities (D3Q27); opposite velocities at (i, i + 1) for odd i.
// Weights: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216 (products of
// the one-dimensional 2/3, 1/6).
__host__ __device__ constexpr int ex(int i) {
  return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13 || i == 19 || i == 21 || i == 23 ||
          i == 26) ? 1
       : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14 || i == 20 || i == 22 || i == 24 ||
          i == 25) ? -1 : 0;
}
__host__ __device__ constexpr int ey(int i) {
  return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17 || i == 19 || i == 21 || i == 24 ||
          i == 25) ? 1
       : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18 || i == 20 || i == 22 || i == 23 ||
          i == 26) ? -1 : 0;
}
__host__ __device__ constexpr int ez(int i) {
  return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18 || i == 19 || i == 22 || i == 23 ||
          i == 25) ? 1
       : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17 || i == 20 || i == 21 || i == 24 ||
          i == 26) ? -1 : 0;
}
// velocity class: 0 rest, 1 axis, 2 edge, 3 corner
__host__ __device__ constexpr int cls3(int i) { return i == 0 ? 0 : (i <= 6 ? 1 : (i <= 18 ? 2 : 3)); }
template <class R> __host__ __device__ constexpr R w3(int q, int i) {
  return q == 27 ? (cls3(i) == 0 ? R(8) / R(27) : cls3(i) == 1 ? R(2) / R(27)
                                                  : cls3(i) == 2 ? R(1) / R(54) : R(1) / R(216))
                 : (cls3(i) == 0 ? R(1) / R(3) : cls3(i) == 1 ? R(1) / R(18) : R(1) / R(36));
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
static_assert(ex(1) == 1 && ex(2) == -1 && ey(3) == 1 && ey(4) == -1 && ez(5) == 1 && ez(6) == -1,
              "axis velocities");
static_assert(ex(7) == 1 && ey(7) == 1 && ex(8) == -1 && ey(8) == -1, "edge pair 7/8");
static_assert(ex(17) == 0 && ey(17) == 1 && ez(17) == -1 && ey(18) == -1 && ez(18) == 1,
              "edge pair 17/18");
static_assert(ex(19) == 1 && ey(19) == 1 && ez(19) == 1 && ex(21) == 1 && ey(21) == 1 && ez(21) == -1 &&
                  ex(23) == 1 && ey(23) == -1 && ez(23) == 1 && ex(25) == -1 && ey(25) == 1 &&
                  ez(25) == 1,
              "corners 19, 21, 23, 25");
static_assert(ex(20) == -1 && ey(20) == -1 && ez(20) == -1 && ex(26) == 1 && ey(26) == -1 &&
                  ez(26) == -1,
              "corners 20, 26");

constexpr uint32_t NODE_SOLID3 = 0x80000000u;  // node word: the node is solid

struct Dom3 {
  void *f[2];          // populations [Q][nz][ny][pitch], deviations
  uint32_t *nodew;     // [nz][ny][pitch]: NODE_SOLID3, or bit i-1 when the
                       // source x - e_i is solid; null without solids
  uint64_t *tstep;
  uint32_t *health;
  double *partials;    // FP64 density partial sums, one per z plane
  double *mass;
  int nx, ny, nz, pitch;
  int storage;         // 0 FP64, 1 FP32, 2 FP16, 3 BF16
  int sr;              // 16-bit storage rounds stochastically
  uint32_t key0, key1; // rounding-bit key
  int tiles_x, tiles_y;  // 64 x 4 node tiles of one z plane
  int trt;               // two relaxation times (else BGK: tau_m = tau)
  double rho0, tau, omega, gx, gy, gz;
  double tau_m, omega_m;  // relaxation of the antisymmetric parts
  float rho0_f, tau_f, omega_f, gx_f, gy_f, gz_f;
  float tau_m_f, omega_m_f;
  // 16-bit storage (collision in the stored scaling): the even-part,
  // second-order and linear coefficients K w, (9/2) K w, 3 K w of the moving
  // directions (K w = 8/9 for all of them), times omega for BGK; the rest
  // population's relaxation factor (omega for BGK, 1 for TRT) and 1 - omega
  float s_cw, s_cq, s_cl, s_om0, keep_f;
  // power law (Sec. 5): flow index, consistency, clamp of tau*, and the TRT
  // magic number (tau_minus then follows the local tau*)
  int pl;  // power-law local tau*
  double pl_n, pl_K, tau_min, tau_max, magic;
  float pl_n_f, pl_K_f, tau_min_f, tau_max_f, magic_f;
  // thermal noise (BGK): k_B T; Philox key (key0, key1)
  int noise;
  double kT;
  float kT_f;
};

template <class R> __device__ __forceinline__ R par3(double a, float b);
template <> __device__ __forceinline__ double par3<double>(double a, float) { return a; }
template <> __device__ __forceinline__ float par3<float>(double, float b) { return b; }
__device__ __forceinline__ float fmr(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmr(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Local relaxation time of the power-law fluid (Sec. 5) from
// A = 3 |Pi_neq|_F / (sqrt(2) rho) (all nine stress components): the shear
// rate is A / tau*, nu* = K gamma_dot^(n-1) and tau* = 1/2 + 3 nu*, so tau*
// is the root of h(t) = t - 1/2 - c t^(1-n), c = 3 K A^(n-1), clamped to
// [tau_min, tau_max].  n = 1: 1/2 + 3 K; n = 1/2: t = s^2 with
// s = (c + sqrt(c^2 + 2)) / 2; otherwise Newton from the bracket end on the
// side where it converges monotonically (tau_max for n < 1, tau_min above).
template <class R> __device__ __forceinline__ R powr3(R a, R b) {
  if constexpr (sizeof(R) == 8) return pow(a, b);
  else return exp2f(b * log2f(a));
}
template <class R> __device__ R tau_power3(const Dom3 &D, R A) {
  const R n = par3<R>(D.pl_n, D.pl_n_f), xi = par3<R>(D.pl_K, D.pl_K_f);
  const R tmin = par3<R>(D.tau_min, D.tau_min_f), tmax = par3<R>(D.tau_max, D.tau_max_f);
  if (n == R(1)) {
    const R t = R(0.5) + R(3) * xi;
    return t < tmin ? tmin : (t > tmax ? tmax : t);
  }
  const bool thinning = n < R(1);
  if (!(A > R(0))) return thinning ? tmax : tmin;
  R t;
  if (n == R(0.5)) {
    const R c = R(3) * xi / sqrt(A);
    const R sr = R(0.5) * (c + sqrt(c * c + R(2)));
    t = sr * sr;
  } else {
    const R c = R(3) * xi * powr3<R>(A, n - R(1));
    const R t0 = thinning ? tmax : tmin;
    const R h0 = t0 - R(0.5) - c * powr3<R>(t0, R(1) - n);
    if (thinning ? !(h0 > R(0)) : !(h0 < R(0))) return t0;
    constexpr int ITERS = sizeof(R) == 8 ? 40 : 12;
    const R tol = sizeof(R) == 8 ? R(1e-15) : R(1e-7);
    t = t0;
#pragma unroll 1
    for (int it = 0; it < ITERS; ++it) {
      const R tp = powr3<R>(t, R(1) - n);
      const R h = t - R(0.5) - c * tp;
      const R dh = R(1) - c * (R(1) - n) * tp / t;
      const R tn = t - h / dh;
      const bool done = fabs(tn - t) <= tol * tn;
      t = tn;
      if (done) break;
    }
  }
  return t < tmin ? tmin : (t > tmax ? tmax : t);
}

// A = 3 |Pi_neq|_F / (sqrt(2) rho) of a node from the pair sums ps_k of its
// deviations (the second moments are even under e -> -e), each class scaled
// back by inv[class]: Pi_neq = sum e e d - drho/3 I - rho u u with
// u = j / rho + g / 2 (the second moment of the equilibrium is rho/3 I +
// rho u u on both lattices).
template <class R, int Q>
__device__ __forceinline__ R shear_measure3(const Dom3 &D, const R *ps, const R (&inv)[4], R drho,
                                            R rho, R irho, R jx, R jy, R jz) {
  R sxx = R(0), syy = R(0), szz = R(0), sxy = R(0), sxz = R(0), syz = R(0);
#pragma unroll
  for (int k = 1; k <= (Q - 1) / 2; ++k) {
    const int i = 2 * k - 1;
    const R v = inv[cls3(i)] * ps[k];
    if (ex(i)) sxx += v;
    if (ey(i)) syy += v;
    if (ez(i)) szz += v;
    if (ex(i) && ey(i)) sxy += R(ex(i) * ey(i)) * v;
    if (ex(i) && ez(i)) sxz += R(ex(i) * ez(i)) * v;
    if (ey(i) && ez(i)) syz += R(ey(i) * ez(i)) * v;
  }
  const R ux = fmr(jx, irho, R(0.5) * par3<R>(D.gx, D.gx_f));
  const R uy = fmr(jy, irho, R(0.5) * par3<R>(D.gy, D.gy_f));
  const R uz = fmr(jz, irho, R(0.5) * par3<R>(D.gz, D.gz_f));
  const R third = drho * (R(1) / R(3));
  const R pxx = sxx - third - rho * ux * ux, pyy = syy - third - rho * uy * uy,
          pzz = szz - third - rho * uz * uz;
  const R pxy = sxy - rho * ux * uy, pxz = sxz - rho * ux * uz, pyz = syz - rho * uy * uz;
  const R fro2 = pxx * pxx + pyy * pyy + pzz * pzz + R(2) * (pxy * pxy + pxz * pxz + pyz * pyz);
  return R(2.1213203435596424) * sqrt(fro2) * irho;  // 3 / sqrt(2)
}

// Storage of the deviations: FP64 and FP32 as they are; the 16-bit formats
// hold d_i K_i with powers of two K (so scaling is exact) near 1 / w_i, which
// keeps the small deviations of the long velocities clear of the FP16
// subnormal range: D3Q19 K = 2, 16, 32 (w K = 2/3, 8/9, 8/9), D3Q27 K = 4,
// 16, 64, 256 (w K = 32/27 for every class); converted with round to
// nearest or the hardware's stochastic rounding.
__host__ __device__ constexpr float scale3(int q, int i) {
  return q == 27 ? (cls3(i) == 0 ? 4.0f : cls3(i) == 1 ? 16.0f : cls3(i) == 2 ? 64.0f : 256.0f)
                 : (cls3(i) == 0 ? 2.0f : cls3(i) == 1 ? 16.0f : 32.0f);
}
template <int ST> struct S3;
template <> struct S3<0> {
  using T = double;
  using R = double;
  static __device__ __forceinline__ R dec(T v, int, int) { return v; }
  static __device__ __forceinline__ T enc(R v, int, int, bool, uint32_t) { return v; }
};
template <> struct S3<1> {
  using T = float;
  using R = float;
  static __device__ __forceinline__ R dec(T v, int, int) { return v; }
  static __device__ __forceinline__ T enc(R v, int, int, bool, uint32_t) { return v; }
};
template <> struct S3<2> {
  using T = uint16_t;
  using R = float;
  static __device__ __forceinline__ R dec(T v, int q, int i) { return lbk::f16_to_f32(v) * (1.0f / scale3(q, i)); }
  static __device__ __forceinline__ R raw(T v) { return lbk::f16_to_f32(v); }
  static __device__ __forceinline__ T enc_raw(R v, bool sr, uint32_t r) {
    return sr ? lbk::f32_to_f16_sr(v, r) : lbk::f32_to_f16_rn(v);
  }
  static __device__ __forceinline__ T enc(R v, int q, int i, bool sr, uint32_t r) {
    return sr ? lbk::f32_to_f16_sr(v * scale3(q, i), r) : lbk::f32_to_f16_rn(v * scale3(q, i));
  }
};
template <> struct S3<3> {
  using T = uint16_t;
  using R = float;
  static __device__ __forceinline__ R dec(T v, int q, int i) { return lbk::bf16_to_f32(v) * (1.0f / scale3(q, i)); }
  static __device__ __forceinline__ R raw(T v) { return lbk::bf16_to_f32(v); }
  static __device__ __forceinline__ T enc_raw(R v, bool sr, uint32_t r) {
    return sr ? lbk::f32_to_bf16_sr(v, r) : lbk::f32_to_bf16_rn(v);
  }
  static __device__ __forceinline__ T enc(R v, int q, int i, bool sr, uint32_t r) {
    return sr ? lbk::f32_to_bf16_sr(v * scale3(q, i), r) : lbk::f32_to_bf16_rn(v * scale3(q, i));
  }
};

// Rounding bits of a node and step: one hash of (node, step, key), spread
// over the directions by the multiplicative hash the D2Q9 sweep uses.
__device__ __forceinline__ uint32_t round_bits3(const Dom3 &D, uint32_t node, uint32_t step) {
  return lbk::mix32(node ^ (lbk::mix32(step ^ D.key0) ^ D.key1));
}

// sqrt(w_i): D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216
template <class R> __device__ __forceinline__ constexpr R sqw3(int q, int i) {
  return q == 27 ? (cls3(i) == 0   ? R(0.544331053951817355154952016601)
                    : cls3(i) == 1 ? R(0.272165526975908677577476008301)
                    : cls3(i) == 2 ? R(0.136082763487954338788738004150)
                                   : R(0.0680413817439771693943690020752))
                 : (cls3(i) == 0   ? R(0.577350269189625764509148780502)
                    : cls3(i) == 1 ? R(0.235702260395515841466948120702)
                                   : R(0.166666666666666666666666666667));
}

// Thermal noise of one collision (Sec. 4, Eqs. NP1-NP2, carried to 3D): the
// D2Q9 method's law, independent unit noise on every mode other than mass
// and momentum scaled by amp = sqrt(3 rho kT omega (2 - omega)), drawn
// without a mode basis.  eta_i = amp sqrt(w_i) xi_i from q unit normals has
// covariance amp^2 W, W = diag(w); taking away its mass and momentum parts,
// zeta_i = eta_i - w_i (S + 3 e_i.V), S = sum eta, V = sum e eta, leaves the
// covariance amp^2 (W - w w^T - 3 (W e)(W e)^T), the same as the mode form.  Philox
// block b of (node, step) gives xi_{6b} .. xi_{6b+5} (three Box-Muller
// pairs, the D2Q9 recipe); FP32 arithmetic takes the hardware transform,
// FP64 the exact one.  With TRT the parts of eta even and odd under
// e -> -e relax with omega and omega_m; each carries its own amplitude,
// mass leaving the even part and momentum the odd one:
// zeta = amp (eta_s - w S) + amp_m (eta_a - 3 w e.V) (orthogonal parts).
template <class R, int Q, bool TRTN>
__device__ __forceinline__ void noise3(const Dom3 &D, uint32_t node, uint32_t step, R rho, R om,
                                       R omm, R z[Q]) {
  constexpr int PAIRS = (Q + 1) / 2;
  float xi[2 * PAIRS];
#pragma unroll
  for (int b = 0; 3 * b < PAIRS; ++b) {
    uint32_t w[4];
    lbk::philox4x32_10(node, step, (uint32_t)b, 0u, D.key0, D.key1, w);
    const uint32_t k[6] = {w[0] >> 11, w[1] >> 11, w[2] >> 11, w[3] >> 11,
                           ((w[0] & 0x7ffu) << 10) | (w[2] & 0x3ffu),
                           ((w[1] & 0x7ffu) << 10) | (w[3] & 0x3ffu)};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int j = 3 * b + p;
      if (j < PAIRS) {
        if constexpr (sizeof(R) == 4) lbk::noise_pair_hw(k[2 * p], k[2 * p + 1], xi[2 * j], xi[2 * j + 1]);
        else lbk::noise_pair(k[2 * p], k[2 * p + 1], xi[2 * j], xi[2 * j + 1]);
      }
    }
  }
  const R kT3 = R(3) * rho * par3<R>(D.kT, D.kT_f);
  const R amp = sqrt(kT3 * om * (R(2) - om));
  if constexpr (TRTN) {
    const R ampm = sqrt(kT3 * omm * (R(2) - omm));
    R S = R(0), Vx = R(0), Vy = R(0), Vz = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      z[i] = sqw3<R>(Q, i) * R(xi[i]);
      S += z[i];
      if (ex(i)) Vx += R(ex(i)) * z[i];
      if (ey(i)) Vy += R(ey(i)) * z[i];
      if (ez(i)) Vz += R(ez(i)) * z[i];
    }
    z[0] = amp * fmr(-w3<R>(Q, 0), S, z[0]);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {  // the pair (i, i + 1), e_{i+1} = -e_i
      const R w = w3<R>(Q, i);
      R eV = R(0);
      if (ex(i)) eV += R(ex(i)) * Vx;
      if (ey(i)) eV += R(ey(i)) * Vy;
      if (ez(i)) eV += R(ez(i)) * Vz;
      const R es = amp * fmr(R(0.5), z[i] + z[i + 1], -w * S);
      const R ea = ampm * fmr(R(0.5), z[i] - z[i + 1], R(-3) * w * eV);
      z[i] = es + ea;
      z[i + 1] = es - ea;
    }
    return;
  }
  // amp sqrt(w) per velocity class (rest, axis, edge, corner): the
  // amplitude enters once, through eta
  const R as[4] = {amp * sqw3<R>(Q, 0), amp * sqw3<R>(Q, 1), amp * sqw3<R>(Q, 7),
                   amp * sqw3<R>(Q, Q - 1)};
  R S = R(0), Vx = R(0), Vy = R(0), Vz = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    z[i] = as[cls3(i)] * R(xi[i]);
    S += z[i];
    if (ex(i)) Vx += R(ex(i)) * z[i];
    if (ey(i)) Vy += R(ey(i)) * z[i];
    if (ez(i)) Vz += R(ez(i)) * z[i];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    R m = S;
    if (ex(i)) m += R(3 * ex(i)) * Vx;
    if (ey(i)) m += R(3 * ey(i)) * Vy;
    if (ez(i)) m += R(3 * ez(i)) * Vz;
    z[i] = fmr(-w3<R>(Q, i), m, z[i]);
  }
}

// BGK or TRT collision of one node in deviation form.  The equilibrium of
// Eq. LB2 with u = J / rho, J = j + rho tau_m g (tau_m = tau for BGK):
// opposite velocities share the even part c and take c +- 3 w (e.J); the
// rest population is delta rho less the others.  BGK relaxes every
// d_i with omega; TRT relaxes the part of (feq - d) symmetric over a pair
// with omega and the antisymmetric part with omega_m (the rest population is
// symmetric).  FP32 arithmetic forms the increment and gives it exactly the
// method's mass (zero) and momentum (rho g) from sums of the small
// increments before the one final rounding, as the D2Q9 sweep does (the
// momentum term of the stored values would otherwise round the body force
// of slow flows with a bias).
// NZ: no noise (0), noise with BGK (1) or with TRT (2)
template <class R, int Q, bool PL, int NZ>
__device__ __forceinline__ void collide3(const Dom3 &D, R d[Q], uint32_t node, uint32_t step) {
  R drho = d[0];
#pragma unroll
  for (int i = 1; i < Q; i += 2) drho += d[i] + d[i + 1];
  R jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const R o = d[i] - d[i + 1];  // e_{i+1} = -e_i
    if (ex(i)) jx += R(ex(i)) * o;
    if (ey(i)) jy += R(ey(i)) * o;
    if (ez(i)) jz += R(ez(i)) * o;
  }
  const R rho = par3<R>(D.rho0, D.rho0_f) + drho;
  const R irho = R(1) / rho;
  // tau: the relaxation time of the force shift (tau_minus for TRT)
  R tau = par3<R>(D.tau_m, D.tau_m_f), om = par3<R>(D.omega, D.omega_f);
  R omm = par3<R>(D.omega_m, D.omega_m_f);
  if constexpr (PL) {
    R ps[(Q - 1) / 2 + 1];
#pragma unroll
    for (int k = 1; k <= (Q - 1) / 2; ++k) ps[k] = d[2 * k - 1] + d[2 * k];
    const R inv[4] = {R(1), R(1), R(1), R(1)};
    const R ts = tau_power3<R>(D, shear_measure3<R, Q>(D, ps, inv, drho, rho, irho, jx, jy, jz));
    om = R(1) / ts;
    if (D.trt) {
      tau = R(0.5) + par3<R>(D.magic, D.magic_f) / (ts - R(0.5));
      omm = R(1) / tau;
    } else {
      tau = ts;
      omm = om;
    }
  }
  const R gx = par3<R>(D.gx, D.gx_f), gy = par3<R>(D.gy, D.gy_f), gz = par3<R>(D.gz, D.gz_f);
  const R rt = rho * tau;
  const R Jx = fmr(rt, gx, jx), Jy = fmr(rt, gy, jy), Jz = fmr(rt, gz, jz);
  const R ux = Jx * irho, uy = Jy * irho, uz = Jz * irho;
  const R q = (R(1.5) * rho) * fmr(ux, ux, fmr(uy, uy, uz * uz));
  const R r45 = R(4.5) * rho;
  R eq[Q];
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const R w = w3<R>(Q, i);
    const R eu = R(ex(i)) * ux + R(ey(i)) * uy + R(ez(i)) * uz;
    const R eJ = R(ex(i)) * Jx + R(ey(i)) * Jy + R(ez(i)) * Jz;
    const R c = w * (drho + fmr(r45 * eu, eu, -q));
    const R l = (R(3) * w) * eJ;
    eq[i] = c + l;
    eq[i + 1] = c - l;
  }
  if constexpr (sizeof(R) == 4) {
    R inc[Q];
    if (D.trt) {
#pragma unroll
      for (int i = 1; i < Q; i += 2) {
        const R a = eq[i] - d[i], b = eq[i + 1] - d[i + 1];
        const R sym = R(0.5) * (a + b), anti = R(0.5) * (a - b);
        inc[i] = fmr(om, sym, omm * anti);
        inc[i + 1] = fmr(om, sym, -(omm * anti));
      }
    } else {
#pragma unroll
      for (int i = 1; i < Q; ++i) inc[i] = om * (eq[i] - d[i]);
    }
    if constexpr (NZ != 0) {
      // the noise has no mass or momentum: the rest population's share
      // follows from the mass balance below, its rounding from the momentum
      // correction
      R z[Q];
      noise3<R, Q, NZ == 2>(D, node, step, rho, om, omm, z);
#pragma unroll
      for (int i = 1; i < Q; ++i) inc[i] += z[i];
    }
    R sx = R(0), sy = R(0), sz = R(0);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      const R o = inc[i] - inc[i + 1];
      if (ex(i)) sx += R(ex(i)) * o;
      if (ey(i)) sy += R(ey(i)) * o;
      if (ez(i)) sz += R(ez(i)) * o;
    }
    const R hx = R(0.5) * fmr(rho, gx, -sx), hy = R(0.5) * fmr(rho, gy, -sy),
            hz = R(0.5) * fmr(rho, gz, -sz);
    inc[1] += hx;
    inc[2] -= hx;
    inc[3] += hy;
    inc[4] -= hy;
    inc[5] += hz;
    inc[6] -= hz;
    R m = R(0);
#pragma unroll
    for (int i = 1; i < Q; i += 2) m += inc[i] + inc[i + 1];
    inc[0] = -m;
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = d[i] + inc[i];
  } else {
    R s = R(0);
#pragma unroll
    for (int i = 1; i < Q; i += 2) s += eq[i] + eq[i + 1];
    eq[0] = drho - s;
    if (D.trt) {
      d[0] = fmr(om, eq[0] - d[0], d[0]);
#pragma unroll
      for (int i = 1; i < Q; i += 2) {
        const R a = eq[i] - d[i], b = eq[i + 1] - d[i + 1];
        const R sym = R(0.5) * (a + b), anti = R(0.5) * (a - b);
        d[i] += fmr(om, sym, omm * anti);
        d[i + 1] += fmr(om, sym, -(omm * anti));
      }
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) d[i] = fmr(om, eq[i] - d[i], d[i]);
    }
    if constexpr (NZ != 0) {
      R z[Q];
      noise3<R, Q, NZ == 2>(D, node, step, rho, om, omm, z);
#pragma unroll
      for (int i = 0; i < Q; ++i) d[i] += z[i];
    }
  }
}

// The same collision for the 16-bit formats, on the stored values d_i K_i
// in FP32.  In that scaling every moving direction has the same K_i w_i
// (8/9 on D3Q19, 32/27 on D3Q27), so its even part is cw (drho - q) +
// cq rho (e.u)^2 and its linear part cl (e.J), one coefficient triple per
// domain (times omega for BGK, so that the relaxation is one fma a
// direction); the rest population takes the mass balance,
// K_0 (omega drho - sum of the others / K_i).  The pair sums and
// differences of the stored values give drho and j and, for TRT, the
// symmetric and antisymmetric parts.  Relaxation is applied to the stored
// values directly (no increment form: the rounding to 16 bits is far
// coarser than the FP32 arithmetic).
template <int Q, bool PL, int NZ>
__device__ __forceinline__ void collide3_scaled(const Dom3 &D, float d[Q], uint32_t node, uint32_t step) {
  constexpr int P = (Q - 1) / 2;  // direction pairs: k covers 2k - 1 and 2k
  float ps[P + 1], pd[P + 1];
#pragma unroll
  for (int k = 1; k <= P; ++k) {
    ps[k] = d[2 * k - 1] + d[2 * k];
    pd[k] = d[2 * k - 1] - d[2 * k];
  }
  // per class (axis, edge, corner): the sums of the pairs' sums, and the
  // momentum parts sum e pd; scaled back by 1 / K of the class
  float sc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  float jc[4][3] = {};
#pragma unroll
  for (int k = 1; k <= P; ++k) {
    const int i = 2 * k - 1, c = cls3(i);
    sc[c] += ps[k];
    if (ex(i)) jc[c][0] += float(ex(i)) * pd[k];
    if (ey(i)) jc[c][1] += float(ey(i)) * pd[k];
    if (ez(i)) jc[c][2] += float(ez(i)) * pd[k];
  }
  constexpr float i0 = 1.0f / scale3(Q, 0), i1 = 1.0f / scale3(Q, 1), i2 = 1.0f / scale3(Q, 7),
                  i3 = 1.0f / scale3(Q, Q - 1);
  float drho = fmr(i0, d[0], fmr(i1, sc[1], i2 * sc[2]));
  float jxyz[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) jxyz[a] = fmr(i1, jc[1][a], i2 * jc[2][a]);
  if constexpr (Q == 27) {
    drho = fmr(i3, sc[3], drho);
#pragma unroll
    for (int a = 0; a < 3; ++a) jxyz[a] = fmr(i3, jc[3][a], jxyz[a]);
  }
  const float rho = D.rho0_f + drho;
  const float irho = __builtin_amdgcn_rcpf(rho);  // 1 ulp: enters only the second-order term
  // the domain's coefficients, or with the power law those of the local tau*
  float tm = D.tau_m_f, cw = D.s_cw, cq = D.s_cq, cl = D.s_cl, om0 = D.s_om0, keep = D.keep_f;
  float om = D.omega_f, omm = D.omega_m_f;
  if constexpr (PL) {
    const float inv[4] = {i0, i1, i2, i3};
    const float ts = tau_power3<float>(
        D, shear_measure3<float, Q>(D, ps, inv, drho, rho, irho, jxyz[0], jxyz[1], jxyz[2]));
    om = 1.0f / ts;
    constexpr float kw = Q == 27 ? 32.0f / 27.0f : 8.0f / 9.0f;
    if (D.trt) {
      tm = 0.5f + D.magic_f / (ts - 0.5f);
      omm = 1.0f / tm;
      cw = kw;
      om0 = 1.0f;
    } else {
      tm = ts;
      cw = om * kw;
      om0 = om;
      keep = 1.0f - om;
    }
    cq = 4.5f * cw;
    cl = 3.0f * cw;
  }
  const float rt = rho * tm;
  const float Jx = fmr(rt, D.gx_f, jxyz[0]), Jy = fmr(rt, D.gy_f, jxyz[1]),
              Jz = fmr(rt, D.gz_f, jxyz[2]);
  const float ux = Jx * irho, uy = Jy * irho, uz = Jz * irho;
  const float q = (1.5f * rho) * fmr(ux, ux, fmr(uy, uy, uz * uz));
  const float b = cw * (drho - q);
  const float a = cq * rho;
  const float ax = a * ux, ay = a * uy, az = a * uz;
  const float lx = cl * Jx, ly = cl * Jy, lz = cl * Jz;
  float c[P + 1], l[P + 1];
  float cs[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // per class: sum of the even parts
#pragma unroll
  for (int k = 1; k <= P; ++k) {
    const int i = 2 * k - 1;
    float eu = 0.0f, aeu = 0.0f, lin = 0.0f;
    if (ex(i)) { eu += float(ex(i)) * ux; aeu += float(ex(i)) * ax; lin += float(ex(i)) * lx; }
    if (ey(i)) { eu += float(ey(i)) * uy; aeu += float(ey(i)) * ay; lin += float(ey(i)) * ly; }
    if (ez(i)) { eu += float(ez(i)) * uz; aeu += float(ez(i)) * az; lin += float(ez(i)) * lz; }
    c[k] = fmr(aeu, eu, b);
    l[k] = lin;
    cs[cls3(i)] += c[k];
  }
  // pair k contributes 2 c_k / K: rest = K0 om0 drho - 2 K0 sum_class cs / K_class
  constexpr float K0 = scale3(Q, 0);
  float others = fmr(i1, cs[1], i2 * cs[2]);
  if constexpr (Q == 27) others = fmr(i3, cs[3], others);
  const float eq0 = fmr(K0 * om0, drho, -(2.0f * K0) * others);
  if (!D.trt) {
    d[0] = fmr(keep, d[0], eq0);
#pragma unroll
    for (int k = 1; k <= P; ++k) {
      d[2 * k - 1] = fmr(keep, d[2 * k - 1], c[k] + l[k]);
      d[2 * k] = fmr(keep, d[2 * k], c[k] - l[k]);
    }
  } else {
    d[0] = fmr(om, eq0 - d[0], d[0]);
#pragma unroll
    for (int k = 1; k <= P; ++k) {
      const float sym = fmr(-0.5f, ps[k], c[k]), anti = fmr(-0.5f, pd[k], l[k]);
      const float t = omm * anti;
      d[2 * k - 1] += fmr(om, sym, t);
      d[2 * k] += fmr(om, sym, -t);
    }
  }
  if constexpr (NZ != 0) {
    float z[Q];
    noise3<float, Q, NZ == 2>(D, node, step, rho, om, omm, z);
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = fmr(scale3(Q, i), z[i], d[i]);
  }
}

// XCD-aware block order: the hardware deals consecutive block ids to the 8
// XCDs in turn; remapped, each XCD walks a contiguous run of tiles, so the
// 128-byte lines that an x-shifted pull shares with the neighbouring tile
// are found in the same L2 (without it the FP32 256^3 sweep read 1.26 x its
// populations).
__device__ __forceinline__ int xcd_order(int bid, int nblocks) {
  constexpr int NX = 8;
  if (nblocks < 2 * NX) return bid;
  const int xcd = bid % NX, local = bid / NX;
  const int per = nblocks / NX, rem = nblocks % NX;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Raw buffer access: the memory unit adds a wave-uniform (scalar) and a
// per-lane byte offset to the buffer's base, so the plane part of every
// address costs no vector instruction.  Word 3 is the raw-buffer format of
// the gfx9 family.
typedef __amdgpu_buffer_rsrc_t Res3;
__device__ __forceinline__ Res3 res3(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
template <class T> __device__ __forceinline__ T ld3(Res3 r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 2)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <class T> __device__ __forceinline__ void st3(Res3 r, uint32_t voff, uint32_t soff, T v) {
  if constexpr (sizeof(T) == 2) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, (int)voff, (int)soff, 0);
  } else if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 0);
  } else {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
  }
}

// One step of every node: 256 threads = a tile of 64 (x) by 4 (y) nodes of
// one z plane; each wave reads 64 consecutive x of a row per population
// plane.  D3Q19: eight waves per SIMD for the FP32 and 16-bit formats (at
// most 64 registers), four for FP64; D3Q27 and the power law: at least four,
// half as many for FP64 (no spills).  A solid node stores zero deviations (every slot is written each
// step and never pulled).  Addressing: each direction pair (i odd, i + 1)
// loads at the pair's first population plane (a wave-uniform offset) plus a
// per-lane byte offset, and stores at its own plane plus the node's offset;
// with WIDE false (Q population planes below 2^32 bytes) these are raw
// buffer accesses, and a pulled population costs one vector add for its
// address.  A bounced link reads the opposite population of the node itself,
// from the same pair base.  SOLIDS false: no node words (no walls or
// obstacles).
// Waves per SIMD the register budget is sized for (FP64 holds twice the
// registers; the power law and the noise take more of them).
constexpr int sweep3_waves(int st, int q, bool pl, bool noise) {
  const int base = st == 0 ? (q == 27 ? 2 : 4) / (pl ? 2 : 1) : (q == 27 || pl ? 4 : 8);
  const int cap = st == 0 ? 2 : 4;
  return noise && base > cap ? cap : base;
}

template <int ST, bool SOLIDS, bool WIDE, int Q, bool PL, int NZ>
__global__ __launch_bounds__(256, sweep3_waves(ST, Q, PL, NZ != 0)) void k_sweep3(const Dom3 *__restrict__ Dp, int kstep) {
  using S = S3<ST>;
  using T = typename S::T;
  using R = typename S::R;
  using Off = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  constexpr Off E = sizeof(T);
  const Dom3 &D = *Dp;
  const int nx = D.nx, ny = D.ny, nz = D.nz, pitch = D.pitch;
  const int per_plane = D.tiles_x * D.tiles_y;
  const int b = xcd_order((int)blockIdx.x, (int)gridDim.x);
  const int z = b / per_plane;
  const int t = b - z * per_plane;
  const int ty = t / D.tiles_x, tx = t - ty * D.tiles_x;
  const int x = tx * 64 + (int)(threadIdx.x & 63);
  const int y = ty * 4 + (int)(threadIdx.x >> 6);
  if (x >= nx || y >= ny) return;
  // state time of the source buffer, made wave-uniform so that the buffer
  // bases stay in scalar registers
  const uint64_t ts = *lbk::gbl(D.tstep);
  const uint64_t T0 =
      (((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(ts >> 32)) << 32) |
       __builtin_amdgcn_readfirstlane((uint32_t)ts)) + (uint64_t)kstep;
  const bool odd = (T0 & 1) != 0;
  const LBK_GLOBAL char *src = lbk::gbl((const char *)(odd ? D.f[1] : D.f[0]));
  LBK_GLOBAL char *dst = lbk::gbl((char *)(odd ? D.f[0] : D.f[1]));
  const Off rowb = (Off)pitch * E, zb = (Off)ny * rowb, popb = (Off)nz * zb;
  const Res3 rs = res3((const void *)src, (uint32_t)(Q * popb));
  const Res3 rd = res3((const void *)dst, (uint32_t)(Q * popb));
  // byte offsets of the source columns and planes x - e_i (rows below)
  const Off xo_m = (Off)(x > 0 ? x - 1 : nx - 1) * E, xo_0 = (Off)x * E,
            xo_p = (Off)(x + 1 < nx ? x + 1 : 0) * E;
  const Off zo_m = (Off)(z > 0 ? z - 1 : nz - 1) * zb, zo_0 = (Off)z * zb,
            zo_p = (Off)(z + 1 < nz ? z + 1 : 0) * zb;
  // 16-bit formats: the stored scaling throughout (collide3_scaled)
  auto in = [](T v, int i) -> R {
    if constexpr (sizeof(T) == 2) return S::raw(v);
    else return S::dec(v, Q, i);
  };
  const Off node = ((Off)z * (Off)ny + (Off)y) * (Off)pitch + (Off)x;
  const Off here = node * E;
  uint32_t w = 0u;
  if constexpr (SOLIDS) w = lbk::gbl(D.nodew)[node];
  R d[Q];
  if (SOLIDS && (w & NODE_SOLID3)) {
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = R(0);
  } else {
    const Off yo_m = (Off)(y > 0 ? y - 1 : ny - 1) * rowb, yo_0 = (Off)y * rowb,
              yo_p = (Off)(y + 1 < ny ? y + 1 : 0) * rowb;
    if constexpr (WIDE)
      d[0] = in(*(const LBK_GLOBAL T *)(src + here), 0);
    else
      d[0] = in(ld3<T>(rs, here, 0u), 0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int lo = (i - 1) | 1;  // the pair's first direction: i odd, or i - 1
      const Off zo = ez(i) > 0 ? zo_m : (ez(i) < 0 ? zo_p : zo_0);
      const Off yo = ey(i) > 0 ? yo_m : (ey(i) < 0 ? yo_p : yo_0);
      const Off xo = ex(i) > 0 ? xo_m : (ex(i) < 0 ? xo_p : xo_0);
      Off off = zo + yo + xo + ((i & 1) ? (Off)0 : popb);
      if constexpr (SOLIDS) {
        // halfway bounce-back: population opp(i) of this node
        const Off bb = (i & 1) ? here + popb : here;
        off = ((w >> (i - 1)) & 1u) ? bb : off;
      }
      if constexpr (WIDE)
        d[i] = in(*(const LBK_GLOBAL T *)(src + (Off)lo * popb + off), i);
      else
        d[i] = in(ld3<T>(rs, off, __builtin_amdgcn_readfirstlane((uint32_t)lo * popb)), i);
    }
    // the noise counter: the unpadded node number and the step this
    // collision produces
    const uint32_t nn = ((uint32_t)z * (uint32_t)ny + (uint32_t)y) * (uint32_t)nx + (uint32_t)x;
    const uint32_t step = (uint32_t)(T0 + 1);
    if constexpr (sizeof(T) == 2) collide3_scaled<Q, PL, NZ>(D, d, nn, step);
    else collide3<R, Q, PL, NZ>(D, d, nn, step);
    if (!(fabs((double)d[0]) < 1e30)) atomicOr(D.health, 1u);
  }
  const uint32_t h = sizeof(T) == 2 && D.sr ? round_bits3(D, (uint32_t)node, (uint32_t)T0) : 0u;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    T v;
    if constexpr (sizeof(T) == 2) v = S::enc_raw(d[i], D.sr, lbk::sr_bits(h, i));
    else v = S::enc(d[i], Q, i, false, 0u);
    if constexpr (WIDE)
      *(LBK_GLOBAL T *)(dst + (Off)i * popb + here) = v;
    else
      st3<T>(rd, here, __builtin_amdgcn_readfirstlane((uint32_t)i * popb), v);
  }
}

// Node words from the solid mask ([nz][ny][pitch] bytes, 1 = solid).
template <int Q>
__global__ __launch_bounds__(256) void k_words3(const Dom3 *__restrict__ Dp, const uint8_t *mask) {
  const Dom3 &D = *Dp;
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long total = (long long)D.nz * D.ny * D.nx;
  if (n >= total) return;
  const int x = (int)(n % D.nx), y = (int)((n / D.nx) % D.ny), z = (int)(n / ((long long)D.nx * D.ny));
  auto at = [&](int a, int b, int c) {
    a = (a + D.nx) % D.nx;
    b = (b + D.ny) % D.ny;
    c = (c + D.nz) % D.nz;
    return mask[((size_t)c * D.ny + b) * D.pitch + a];
  };
  uint32_t w = 0;
  if (at(x, y, z)) {
    w = NODE_SOLID3;
  } else {
#pragma unroll
    for (int i = 1; i < Q; ++i)
      if (at(x - ex(i), y - ey(i), z - ez(i))) w |= 1u << (i - 1);
  }
  D.nodew[((size_t)z * D.ny + y) * D.pitch + x] = w;
}

// Equilibrium of the given fields (or rest) as the initial post-collision
// state, after one collision (as the D2Q9 domains start).  Nodes n0 .. n0 +
// cnt - 1; the fields (or null: rest) hold those nodes, [cnt] each.
template <int ST, int Q>
__global__ __launch_bounds__(256) void k_init3(const Dom3 *__restrict__ Dp, const double *rho_f,
                                               const double *ux_f, const double *uy_f,
                                               const double *uz_f, long long n0, long long cnt) {
  using S = S3<ST>;
  using T = typename S::T;
  using R = typename S::R;
  const Dom3 &D = *Dp;
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= cnt) return;
  const long long n = n0 + k;
  const int x = (int)(n % D.nx), y = (int)((n / D.nx) % D.ny), z = (int)(n / ((long long)D.nx * D.ny));
  const size_t plane = (size_t)D.nz * D.ny * D.pitch;
  const size_t here = ((size_t)z * D.ny + y) * D.pitch + x;
  T *dst = (T *)D.f[*D.tstep & 1];
  const bool solid = D.nodew && (D.nodew[here] & NODE_SOLID3);
  R d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = R(0);
  if (rho_f && !solid) {
    const double r = rho_f[k], vx = ux_f[k], vy = uy_f[k], vz = uz_f[k];
    const double uu = vx * vx + vy * vy + vz * vz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double w = w3<double>(Q, i);
      const double eu = ex(i) * vx + ey(i) * vy + ez(i) * vz;
      d[i] = (R)(w * ((r - D.rho0) + r * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu)));
    }
  }
  if (!solid) {
    const uint32_t nn = (uint32_t)n, step = (uint32_t)*D.tstep;
    if (D.noise && D.trt) {
      if (D.pl) collide3<R, Q, true, 2>(D, d, nn, step);
      else collide3<R, Q, false, 2>(D, d, nn, step);
    } else if (D.noise) {
      if (D.pl) collide3<R, Q, true, 1>(D, d, nn, step);
      else collide3<R, Q, false, 1>(D, d, nn, step);
    } else {
      if (D.pl) collide3<R, Q, true, 0>(D, d, nn, step);
      else collide3<R, Q, false, 0>(D, d, nn, step);
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) dst[(size_t)i * plane + here] = S::enc(d[i], Q, i, false, 0u);
}

// rho and u = j/rho + g/2 of the pre-collision state, recovered from f*:
// collision keeps rho and adds rho g to j.
// Nodes n0 .. n0 + cnt - 1 (x fastest) into out [4][cnt].
template <int ST, int Q>
__global__ __launch_bounds__(256) void k_moments3(const Dom3 *__restrict__ Dp, double *out,
                                                  long long n0, long long cnt) {
  using S = S3<ST>;
  using T = typename S::T;
  const Dom3 &D = *Dp;
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= cnt) return;
  const long long n = n0 + k, total = cnt;
  const int x = (int)(n % D.nx), y = (int)((n / D.nx) % D.ny), z = (int)(n / ((long long)D.nx * D.ny));
  const size_t plane = (size_t)D.nz * D.ny * D.pitch;
  const size_t here = ((size_t)z * D.ny + y) * D.pitch + x;
  if (D.nodew && (D.nodew[here] & NODE_SOLID3)) {
    out[k] = out[total + k] = out[2 * total + k] = out[3 * total + k] = 0.0;
    return;
  }
  const T *src = (const T *)D.f[*D.tstep & 1];
  double dr = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double v = (double)S::dec(src[(size_t)i * plane + here], Q, i);
    dr += v;
    jx += ex(i) * v;
    jy += ey(i) * v;
    jz += ez(i) * v;
  }
  const double rho = D.rho0 + dr;
  out[k] = rho;
  out[total + k] = jx / rho - 0.5 * D.gx;
  out[2 * total + k] = jy / rho - 0.5 * D.gy;
  out[3 * total + k] = jz / rho - 0.5 * D.gz;
}

// Populations of nodes n0 .. n0 + cnt - 1 as FP64 deviations, out [Q][cnt].
template <int ST, int Q>
__global__ __launch_bounds__(256) void k_export3(const Dom3 *__restrict__ Dp, double *out,
                                                 long long n0, long long cnt) {
  using S = S3<ST>;
  using T = typename S::T;
  const Dom3 &D = *Dp;
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= cnt) return;
  const long long n = n0 + k;
  const int x = (int)(n % D.nx), y = (int)((n / D.nx) % D.ny), z = (int)(n / ((long long)D.nx * D.ny));
  const size_t plane = (size_t)D.nz * D.ny * D.pitch;
  const size_t here = ((size_t)z * D.ny + y) * D.pitch + x;
  const T *src = (const T *)D.f[*D.tstep & 1];
#pragma unroll
  for (int i = 0; i < Q; ++i)
    out[(size_t)i * cnt + k] = (double)S::dec(src[(size_t)i * plane + here], Q, i);
}

// FP64 density sum: block z sums plane z in a fixed order; one wave adds the
// planes.  Latches a non-finite total.
template <int ST, int Q>
__global__ __launch_bounds__(256) void k_mass3_partial(const Dom3 *__restrict__ Dp) {
  using S = S3<ST>;
  using T = typename S::T;
  __shared__ double red[4];
  const Dom3 &D = *Dp;
  const int z = (int)blockIdx.x;
  const size_t plane = (size_t)D.nz * D.ny * D.pitch;
  const T *src = (const T *)D.f[*D.tstep & 1];
  double acc = 0.0;
  for (int y = 0; y < D.ny; ++y)
    for (int x = (int)threadIdx.x; x < D.nx; x += 256) {
      const size_t here = ((size_t)z * D.ny + y) * D.pitch + x;
      if (D.nodew && (D.nodew[here] & NODE_SOLID3)) continue;
      double r = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) r += (double)S::dec(src[(size_t)i * plane + here], Q, i);
      acc += D.rho0 + r;
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) D.partials[z] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(64) void k_mass3_final(const Dom3 *__restrict__ Dp) {
  const Dom3 &D = *Dp;
  double s = 0.0;
  for (int i = (int)threadIdx.x; i < D.nz; i += 64) s += D.partials[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) {
    *D.mass = s;
    if (!(fabs(s) < 1e300)) atomicOr(D.health, 1u);
  }
}

__global__ void k_advance3(const Dom3 *__restrict__ Dp, int n) { *Dp->tstep += (uint64_t)n; }

}  // namespace lbk3
