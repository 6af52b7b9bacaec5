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
template <class R, int PLM>
__device__ __forceinline__ R powerlaw_tau(const DevDomain &D, const R d[9], R drho, R rho, R irho,
                                          R jx, R jy) {
  const R gx = par<R>(D.gx, D.gx_f), gy = par<R>(D.gy, D.gy_f);
  const R ux = jx * irho + R(0.5) * gx, uy = jy * irho + R(0.5) * gy;
  const R third = drho * (R(1) / R(3));
  const R sxx = (d[1] + d[3]) + ((d[5] + d[6]) + (d[7] + d[8]));
  const R syy = (d[2] + d[4]) + ((d[5] + d[6]) + (d[7] + d[8]));
  const R sxy = (d[5] - d[6]) + (d[7] - d[8]);
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

// BGK collision of one node (deviations in, deviations out), step `step`, in
// arithmetic type R.  The equilibrium of Eq. LB2 with u = j/rho + tau g is
// evaluated in a form whose mass and momentum do not depend on how the
// lattice constants round: the linear term is built from J = j + rho tau g
// with coefficients L1 ~ 1/3, L5 = (1 - 2 L1)/4 (so 2 L1 + 4 L5 = 1 exactly),
// opposite directions share one even part c and take c +- (linear term), and
// the rest population is delta_rho minus the other eight.  Algebraically this
// is Eq. LB2; in FP32 it removes a systematic O(1e-8) momentum error per step
// that would otherwise bias slowly accelerating flows.
template <int ST, int FEAT, int PLM, class R>
__device__ __forceinline__ void collide_node(const DevDomain &D, R d[9], uint32_t node,
                                             uint32_t step) {
  const R drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
  const R jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
  const R jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
  const R rho = par<R>(D.rho0, D.rho0_f) + drho;
  const R irho = R(1) / rho;
  R tau, om;
  if constexpr ((FEAT & F_POWER) != 0) {
    tau = powerlaw_tau<R, PLM>(D, d, drho, rho, irho, jx, jy);
    om = R(1) / tau;
  } else {
    tau = par<R>(D.tau, D.tau_f);
    om = par<R>(D.omega, D.omega_f);
  }
  const R Jx = jx + rho * tau * par<R>(D.gx, D.gx_f);
  const R Jy = jy + rho * tau * par<R>(D.gy, D.gy_f);
  const R ux = Jx * irho, uy = Jy * irho;
  const R W1 = R(1) / R(9), W5 = R(0.25) * W1;
  const R L1 = R(1) / R(3), L5 = (R(1) - R(2) * L1) * R(0.25);
  const R q = R(1.5) * rho * (ux * ux + uy * uy);
  const R r45 = R(4.5) * rho;
  const R sp = ux + uy, sm = uy - ux;
  const R cxx = W1 * (drho + (r45 * ux * ux - q)), cyy = W1 * (drho + (r45 * uy * uy - q));
  const R cpp = W5 * (drho + (r45 * sp * sp - q)), cmm = W5 * (drho + (r45 * sm * sm - q));
  const R lx = L1 * Jx, ly = L1 * Jy, lp = L5 * (Jx + Jy), lm = L5 * (Jy - Jx);
  R eq[9];
  eq[0] = drho - R(2) * ((cxx + cyy) + (cpp + cmm));
  eq[1] = cxx + lx;
  eq[3] = cxx - lx;
  eq[2] = cyy + ly;
  eq[4] = cyy - ly;
  eq[5] = cpp + lp;
  eq[7] = cpp - lp;
  eq[6] = cmm + lm;
  eq[8] = cmm - lm;
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i] = d[i] + om * (eq[i] - d[i]);

  if constexpr ((FEAT & F_NOISE) != 0) {
    float th[6];
    noise_normals(D.key0, D.key1, node, step, th);
    // Theta_k / sqrt(w_k) with w_k = 4, 4/9, 1/9, 2/3, 2/3, 16 (Table t1)
    const R t3 = R(th[0]) * R(0.5), t4 = R(th[1]) * R(1.5), t5 = R(th[2]) * R(3);
    const R t6 = R(th[3]) * R(1.2247448713915890491), t7 = R(th[4]) * R(1.2247448713915890491);
    const R t8 = R(th[5]) * R(0.25);
    const R amp = sqrt(rho * par<R>(D.kT, D.kT_f) * om * (R(2) - om) * R(3));
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const R z = R(basis_poly(3, i)) * t3 + R(basis_poly(4, i)) * t4 + R(basis_poly(5, i)) * t5 +
                  R(basis_poly(6, i)) * t6 + R(basis_poly(7, i)) * t7 + R(basis_poly(8, i)) * t8;
      const R wi = i == 0 ? R(4) * W1 : (i <= 4 ? W1 : W5);  // exact ratios 4 : 1 : 1/4
      d[i] += amp * wi * z;
    }
  }
}

template <int ST, class R>
__device__ __forceinline__ void store_node(const DevDomain &D, typename Store<ST>::T *dst,
                                           size_t plane, uint32_t off, const R d[9],
                                           uint32_t node, uint32_t step) {
  using S = Store<ST>;
  using RS = typename S::R;
  if constexpr (ST == ST_F16 || ST == ST_BF16) {
    if (D.feat & F_STOCH) {
      const uint32_t h = mix32(node * 0x9E3779B1u ^ mix32(step ^ D.key0) ^ D.key1);
#pragma unroll
      for (int i = 0; i < 9; ++i) S::put(dst + i * plane, off, i, (RS)d[i], sr_bits(h, i) | 1u);
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) S::put(dst + i * plane, off, i, (RS)d[i], 0u);
}

// One mirrored value, rounded like the node's own slot of the same direction.
template <int ST, class R>
__device__ __forceinline__ void store_one(const DevDomain &D, typename Store<ST>::T *p, uint32_t off,
                                          int dir, R v, uint32_t node, uint32_t step) {
  using S = Store<ST>;
  using RS = typename S::R;
  if constexpr (ST == ST_F16 || ST == ST_BF16) {
    if (D.feat & F_STOCH) {
      const uint32_t h = mix32(node * 0x9E3779B1u ^ mix32(step ^ D.key0) ^ D.key1);
      S::put(p, off, dir, (RS)v, sr_bits(h, opp(dir)) | 1u);
      return;
    }
  }
  S::put(p, off, dir, (RS)v, 0u);
}

// Arithmetic type: FP64 for FP64 storage or when wide arithmetic is chosen,
// FP32 otherwise.
template <int ST, int WIDE>
using CompT = typename std::conditional<ST == ST_F64 || WIDE != 0, double, float>::type;

// Rows a thread loads before it computes: 16-bit storage moves half the bytes
// per load, so it keeps more rows in flight to cover memory latency.
template <int ST> constexpr int rows_in_flight() { return ST == ST_F16 || ST == ST_BF16 ? 4 : 2; }

// Pull of one node.  Every direction loads the neighbour's slot at x - e_i:
// where that neighbour is solid, its slot holds this node's own opposite
// population, written there by the previous step's store (halfway
// bounce-back by mirror writes); where the pull crosses a particle surface,
// the slot holds the moving-wall bounced value, put there by the particle
// pre-pass (k_link_swap).  So the loads have no data-dependent address.
// Index walls of label-free domains select the node's own slot directly.
template <int ST, int FEAT, class R>
__device__ __forceinline__ uint32_t pull_node(const DevDomain &D, const typename Store<ST>::T *src,
                                              size_t plane, int y, uint32_t here, bool has_lab,
                                              const int (&col)[3], const bool (&col_out)[3],
                                              const bool (&col_wall)[3], R (&d)[9]) {
  using S = Store<ST>;
  const int ny = D.ny, pitch = D.pitch;
  const bool pery = D.bc_y == BC_PERIODIC, wally = D.bc_y == BC_WALL;
  int row[3];
  bool row_out[3], row_wall[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int rr = y + 1 - k;  // k = 0 -> y+1 (source of cy = -1), k = 2 -> y-1
    bool out = false;
    if (rr < 0) { if (pery) rr += ny; else out = true; }
    else if (rr >= ny) { if (pery) rr -= ny; else out = true; }
    row[k] = (out ? y : rr) * pitch;
    row_out[k] = out;
    row_wall[k] = wally && (rr == 0 || rr == ny - 1);
  }
  uint32_t unknown = 0;
  d[0] = (R)S::load(src, here, 0);
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int kc = 1 + cx(i), kr = 1 + cy(i);
    const bool out = col_out[kc] || row_out[kr];
    const uint32_t so = (uint32_t)row[kr] + (uint32_t)col[kc];
    const bool own = out || (!has_lab && (col_wall[kc] || row_wall[kr]));
    d[i] = (R)S::load(src + (own ? opp(i) : i) * plane, own ? here : so, i);
    if (out) unknown |= 1u << i;
  }
  return unknown;
}

// 256 threads.  The plain and obstacle variants are held to at least 5 waves
// per SIMD (enough loads in flight to cover memory latency, no spills); the
// noise and power-law variants keep the compiler's register choice.
template <int FEAT, int WIDE> constexpr int sweep_min_waves() {
  return (FEAT & (F_NOISE | F_POWER)) == 0 && WIDE == 0 ? 5 : 1;
}

template <int ST, int FEAT, int PLM, int WIDE>
__global__ __launch_bounds__(256, (sweep_min_waves<FEAT, WIDE>())) void k_sweep(const DevDomain *__restrict__ doms,
                                               const int *__restrict__ prefix, int ndom,
                                               int kstep) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = CompT<ST, WIDE>;
  constexpr bool LABELS = (FEAT & F_LABELS) != 0;
  constexpr int U = rows_in_flight<ST>();

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
  const int ybase = tyi * rows_pass * npt + (int)threadIdx.x / tw;

  const uint64_t T0 = *gbl(D.tstep) + (uint64_t)kstep;  // state time of the source buffer
  const uint32_t step = (uint32_t)(T0 + 1);
  void *const f0 = D.f[0];
  void *const f1 = D.f[1];
  const T *__restrict__ src = (const T *)((T0 & 1) ? f1 : f0);
  T *__restrict__ dst = (T *)((T0 & 1) ? f0 : f1);
  const size_t plane = (size_t)ny * pitch;
  bool bad = false;  // non-finite density seen by this thread
  const bool perx = D.bc_x == BC_PERIODIC, wallx = D.bc_x == BC_WALL;
  const bool wally = D.bc_y == BC_WALL;
  const bool pressx = D.bc_x == BC_PRESSURE;
  // a batch may mix domains with and without a label plane
  const bool has_lab = LABELS && D.label != nullptr;

  // columns x-1, x, x+1 (index by 1 - cx)
  int col[3];
  bool col_out[3], col_wall[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int c = x + 1 - k;  // k = 0 -> x+1 (source of cx = -1), k = 2 -> x-1 (cx = +1)
    bool out = false;
    if (c < 0) { if (perx) c += nx; else out = true; }
    else if (c >= nx) { if (perx) c -= nx; else out = true; }
    col[k] = out ? x : c;
    col_out[k] = out;
    col_wall[k] = wallx && (c == 0 || c == nx - 1);
  }

#pragma unroll 1
  for (int r0 = 0; r0 < npt; r0 += U) {
    R d[U][9];
    uint32_t unk[U];
    uint16_t nw[U];
    bool act[U];
    // phase 1: every load of the row group, branch-free and none depending on
    // another, so they are all in flight together; rows past the tile or the
    // domain load from a clamped valid row and are discarded
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int yr = ybase + (r0 + u) * rows_pass;
      const bool valid = r0 + u < npt && yr < ny;
      const int y = valid ? yr : ny - 1;
      const uint32_t here = (uint32_t)y * pitch + x;
      nw[u] = (LABELS && has_lab) ? gbl(D.nodew)[here] : (uint16_t)0;
      const bool wall = !(LABELS && has_lab) &&
                        ((wally && (y == 0 || y == ny - 1)) || (wallx && (x == 0 || x == nx - 1)));
      act[u] = valid && !wall;
      unk[u] = pull_node<ST, FEAT, R>(D, src, plane, y, here, LABELS && has_lab, col, col_out,
                                      col_wall, d[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!act[u] || (nw[u] & NODE_SOLID)) continue;
      const int y = ybase + (r0 + u) * rows_pass;
      const uint32_t here = (uint32_t)y * pitch + x;
      if (pressx && unk[u]) {
        // 2/3 + 2 (1/6) = 1 exactly in the chosen constants
        const R half = R(0.5), third2 = R(2) / R(3), sixth = (R(1) - third2) * R(0.5);
        R *e = d[u];
        if (x == 0) {
          const R s = e[0] + e[2] + e[4] + R(2) * (e[3] + e[6] + e[7]);
          const R rux = (par<R>(D.rho_in, D.rho_in_f) - par<R>(D.rho0, D.rho0_f)) - s;
          e[1] = e[3] + third2 * rux;
          e[5] = e[7] - half * (e[2] - e[4]) + sixth * rux;
          e[8] = e[6] + half * (e[2] - e[4]) + sixth * rux;
        } else {
          const R s = e[0] + e[2] + e[4] + R(2) * (e[1] + e[5] + e[8]);
          const R rux = s - (par<R>(D.rho_out, D.rho_out_f) - par<R>(D.rho0, D.rho0_f));
          e[3] = e[1] - third2 * rux;
          e[7] = e[5] + half * (e[2] - e[4]) - sixth * rux;
          e[6] = e[8] - half * (e[2] - e[4]) - sixth * rux;
        }
      }
      const uint32_t node = (uint32_t)y * (uint32_t)nx + (uint32_t)x;
      collide_node<ST, FEAT, PLM, R>(D, d[u], node, step);
      const R drho = ((d[u][0] + d[u][1]) + (d[u][2] + d[u][3])) +
                     ((d[u][4] + d[u][5]) + (d[u][6] + d[u][7])) + d[u][8];
      bad = bad || !(fabs(drho) < R(1e30));
      store_node<ST, R>(D, dst, plane, here, d[u], node, step);
      if (LABELS && (nw[u] & 0xffu)) {
        // mirror writes: the pull along i from the solid source x - e_i will
        // read this node's post-collision opposite population there
#pragma unroll
        for (int i = 1; i < 9; ++i) {
          if (!((nw[u] >> (i - 1)) & 1u)) continue;
          int sy = y - cy(i);
          sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
          const uint32_t so = (uint32_t)sy * pitch + (uint32_t)col[1 + cx(i)];
          store_one<ST, R>(D, dst + i * plane, so, i, d[u][opp(i)], node, step);
        }
      }
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
      d[i] = wgt<R>(i) * (A + rho * (eu + R(0.5) * eu * eu));
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
