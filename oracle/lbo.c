/*
 * lbo.c -- CPU oracle (FP64) for the D2Q9 lattice-Boltzmann method of
 * arXiv:2006.12910.  TEST INFRASTRUCTURE ONLY: used by the tests, the smoke
 * check and the benchmark's CPU-baseline leg, never by the library.
 *
 * Written from the paper's equations; see lbo.h for the step order.  The code
 * is deliberately plain: full populations f (not deviations), two arrays
 * (pre-collision f and post-collision f*), one loop per step of the method, no
 * fusion.  Build flags: -O2 -fno-fast-math -ffp-contract=off.
 */
#include "lbo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- D2Q9 lattice (Sec. 2): e_0 = 0, e_1..4 axis unit vectors at angles
 * (i-1) pi/2, e_5..8 diagonals at angles (2i-9) pi/4; weights 4/9, 1/9, 1/36. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#define CS2 (1.0 / 3.0)

#define MAXP 256

struct lbo_sim {
  lbo_params p;
  int nx, ny;
  int64_t t;
  double *f;      /* pre-collision f(t), [9][ny][nx]   */
  double *fs;     /* post-collision f*(t)              */
  double *fn;     /* streamed f(t+1)                   */
  uint8_t *solid; /* static solids incl. wall rows/cols */
  uint8_t *label; /* 0 fluid, 1 solid, 2+p particle    */
  int np;
  lbo_particle part[MAXP];
  double fcu[MAXP][3];  /* covered/uncovered force + torque for the next step */
  double flink[MAXP][3];     /* exterior-side link force + torque (Eq. MP1)      */
  double flink_int[MAXP][3]; /* interior-side exchange, diagnostic only          */
  double basis[9][9];   /* chi_ki (Table t1), [k][i] */
};

#define IDX(s, i, x, y) (((size_t)(i) * (s)->ny + (y)) * (s)->nx + (x))

/* ---------------------------------------------------------------------- */
/* Noise generator: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11),    */
/* Box-Muller (1958) with this file's own single-precision log / sincos.   */

static uint32_t mulhilo(uint32_t a, uint32_t b, uint32_t *hi) {
  uint64_t prod = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(prod >> 32);
  return (uint32_t)prod;
}

void lbo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  /* round multipliers and Weyl key increments as published by Salmon et al. */
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint32_t hi0, hi1;
    uint32_t lo0 = mulhilo(M0, c0, &hi0);
    uint32_t lo1 = mulhilo(M1, c2, &hi1);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

static float bits_to_float(uint32_t b) {
  float f;
  memcpy(&f, &b, 4);
  return f;
}
static uint32_t float_to_bits(float f) {
  uint32_t b;
  memcpy(&b, &f, 4);
  return b;
}

/* Natural log of a normal float in (0, 1]: exponent split u = m 2^e with
 * m in [sqrt(1/2), sqrt(2)], then ln m = 2 atanh(s), s = (m-1)/(m+1), by its
 * power series to s^11 (Horner steps as fused multiply-adds); ln 2 is split
 * hi + lo (Cody & Waite) so that e*hi is exact.  Every operation is a single
 * IEEE float operation (fmaf: one rounding) in a fixed order. */
float lbo_logf(float u) {
  uint32_t b = float_to_bits(u);
  int e = (int)((b >> 23) & 0xffu) - 127;
  float m = bits_to_float((b & 0x007fffffu) | 0x3f800000u);
  if (m > 1.41421354f) {
    m = m * 0.5f;
    e = e + 1;
  }
  float s = (m - 1.0f) / (m + 1.0f);
  float s2 = s * s;
  float poly = 1.0f / 11.0f;
  poly = fmaf(poly, s2, 1.0f / 9.0f);
  poly = fmaf(poly, s2, 1.0f / 7.0f);
  poly = fmaf(poly, s2, 1.0f / 5.0f);
  poly = fmaf(poly, s2, 1.0f / 3.0f);
  poly = fmaf(poly, s2, 1.0f);
  float lnm = (s + s) * poly;
  const float LN2_HI = 0.693145751953125f;      /* 45426 / 65536              */
  const float LN2_LO = 1.42860682030941723e-6f; /* ln 2 - LN2_HI, rounded     */
  float fe = (float)e;
  return fmaf(fe, LN2_HI, fmaf(fe, LN2_LO, lnm));
}

/* sin and cos of 2 pi u for u a multiple of 2^-22 in (0, 1): exact reduction
 * to a quadrant q and a remainder r in [-1/8, 1/8], then Taylor series of sin
 * (to a^9) and cos (to a^10) at a = 2 pi r, |a| <= pi/4, Horner steps as
 * fused multiply-adds. */
void lbo_sincos2pi(float u, float *sn, float *cs) {
  int q = (int)(u * 4.0f);
  float r = u - 0.25f * (float)q;
  if (r > 0.125f) {
    r = r - 0.25f;
    q = q + 1;
  }
  const float TWO_PI = 6.28318530717958647692f;
  float a = r * TWO_PI;
  float a2 = a * a;
  float ps = 1.0f / 362880.0f;
  ps = fmaf(ps, a2, -1.0f / 5040.0f);
  ps = fmaf(ps, a2, 1.0f / 120.0f);
  ps = fmaf(ps, a2, -1.0f / 6.0f);
  float sa = fmaf(a * a2, ps, a);
  float pc = -1.0f / 3628800.0f;
  pc = fmaf(pc, a2, 1.0f / 40320.0f);
  pc = fmaf(pc, a2, -1.0f / 720.0f);
  pc = fmaf(pc, a2, 1.0f / 24.0f);
  pc = fmaf(pc, a2, -0.5f);
  float ca = fmaf(a2, pc, 1.0f);
  switch (q & 3) {
    case 0: *sn = sa;  *cs = ca;  break;
    case 1: *sn = ca;  *cs = -sa; break;
    case 2: *sn = -sa; *cs = -ca; break;
    default: *sn = -ca; *cs = sa; break;
  }
}

/* uniform in (0,1) from a 21-bit integer: (2k+1) 2^-22, exact in float */
static float unif21(uint32_t k) { return (float)(2u * k + 1u) * (1.0f / 4194304.0f); }

static void box_muller(uint32_t kr, uint32_t ka, float *z0, float *z1) {
  float ur = unif21(kr), ua = unif21(ka);
  float l = lbo_logf(ur);
  float rad = sqrtf(-2.0f * l);
  float sn, cs;
  lbo_sincos2pi(ua, &sn, &cs);
  *z0 = rad * cs;
  *z1 = rad * sn;
}

/* Six standard normals from one Philox4x32-10 block: counter
 * (node, step, block, 0), key (lo32(seed), hi32(seed) ^ domain_id).  The
 * 128 output bits give six 21-bit integers: the top 21 bits of w0..w3, and
 * two built from the low bits, (w0 & 0x7ff) << 10 | (w2 & 0x3ff) and
 * (w1 & 0x7ff) << 10 | (w3 & 0x3ff).  Pairs (w0,w1), (w2,w3) and the two
 * low-bit words feed three Box-Muller transforms (radius, angle). */
void lbo_normals_block(uint64_t seed, uint32_t domain_id, uint32_t node, uint32_t step,
                       uint32_t block, float out[6]) {
  uint32_t ctr[4] = {node, step, block, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ domain_id};
  uint32_t w[4];
  lbo_philox4x32_10(ctr, key, w);
  uint32_t a0 = w[0] >> 11, a1 = w[1] >> 11, a2 = w[2] >> 11, a3 = w[3] >> 11;
  uint32_t b0 = ((w[0] & 0x7ffu) << 10) | (w[2] & 0x3ffu);
  uint32_t b1 = ((w[1] & 0x7ffu) << 10) | (w[3] & 0x3ffu);
  box_muller(a0, a1, &out[0], &out[1]);
  box_muller(a2, a3, &out[2], &out[3]);
  box_muller(b0, b1, &out[4], &out[5]);
}

/* Theta_3..Theta_8 of Eq. NP2 for one node and step: block 0. */
void lbo_normals(uint64_t seed, uint32_t domain_id, uint32_t node, uint32_t step,
                 float out[6]) {
  lbo_normals_block(seed, domain_id, node, step, 0u, out);
}

void lbo_normals_bulk(uint64_t seed, uint32_t domain_id, uint32_t step, uint32_t node0,
                      uint32_t count, float *out) {
  for (uint32_t n = 0; n < count; ++n) lbo_normals(seed, domain_id, node0 + n, step, out + 6 * (size_t)n);
}

/* ---------------------------------------------------------------------- */
/* Table t1: the nine D2Q9 basis polynomials e_ki of the reduced velocity
 * e_i, their lengths w_k = sum_i omega_i e_ki^2, chi_ki = e_ki / sqrt(w_k). */
static void build_basis(double chi[9][9]) {
  for (int i = 0; i < 9; ++i) {
    double ex = EX[i], ey = EY[i], e2 = ex * ex + ey * ey;
    double ek[9];
    ek[0] = 1.0;
    ek[1] = ex;
    ek[2] = ey;
    ek[3] = 3.0 * e2 - 2.0;
    ek[4] = 2.0 * ex * ex - e2;
    ek[5] = ex * ey;
    ek[6] = (3.0 * e2 - 4.0) * ex;
    ek[7] = (3.0 * e2 - 4.0) * ey;
    ek[8] = 9.0 * e2 * e2 - 15.0 * e2 + 2.0;
    for (int k = 0; k < 9; ++k) chi[k][i] = ek[k];
  }
  for (int k = 0; k < 9; ++k) {
    double wk = 0.0;
    for (int i = 0; i < 9; ++i) wk += W[i] * chi[k][i] * chi[k][i];
    double r = sqrt(wk);
    for (int i = 0; i < 9; ++i) chi[k][i] /= r;
  }
}

/* ---------------------------------------------------------------------- */
/* Equilibrium, Eq. LB2 with c_s^2 = 1/3. */
static double feq(int i, double rho, double ux, double uy) {
  double eu = EX[i] * ux + EY[i] * uy;
  double uu = ux * ux + uy * uy;
  return W[i] * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* Power-law relaxation time (Sec. 5).  The shear rate follows from the
 * non-equilibrium stress Pi = sum e e (f - feq(rho, j/rho + g/2)):
 * gamma_dot = A / tau with A = 3 |Pi|_F / (sqrt(2) rho); the viscosity
 * nu* = xi gamma_dot^(n-1) (Eq. nn4 with kappa = 2^(n-1)) and tau* = 1/2 + 3 nu*
 * make tau* the root of h(tau) = tau - 1/2 - 3 xi A^(n-1) tau^(1-n), found by
 * Newton from the bracket end on the side where h keeps its curvature, then
 * clamped to [tau_min, tau_max]. */
static double powerlaw_tau(const lbo_params *p, const double *fl, double rho, double jx,
                           double jy) {
  double n = p->n_index, xi = p->K;
  if (n == 1.0) {
    double t = 0.5 + 3.0 * xi;
    return t < p->tau_min ? p->tau_min : (t > p->tau_max ? p->tau_max : t);
  }
  double ux = jx / rho + 0.5 * p->gx, uy = jy / rho + 0.5 * p->gy;
  double pxx = 0, pyy = 0, pxy = 0;
  for (int i = 0; i < 9; ++i) {
    double d = fl[i] - feq(i, rho, ux, uy);
    pxx += EX[i] * EX[i] * d;
    pyy += EY[i] * EY[i] * d;
    pxy += EX[i] * EY[i] * d;
  }
  double fro = sqrt(pxx * pxx + pyy * pyy + 2.0 * pxy * pxy);
  double A = 3.0 * fro / (sqrt(2.0) * rho);
  double tmin = p->tau_min, tmax = p->tau_max;
  if (A == 0.0) return n < 1.0 ? tmax : tmin;
  double c = 3.0 * xi * pow(A, n - 1.0);
#define HFUN(tt) ((tt) - 0.5 - c * pow((tt), 1.0 - n))
  double t;
  if (n < 1.0) {
    if (HFUN(tmax) <= 0.0) return tmax;
    t = tmax;
  } else {
    if (HFUN(tmin) >= 0.0) return tmin;
    t = tmin;
  }
  for (int it = 0; it < 200; ++it) {
    double h = HFUN(t);
    double dh = 1.0 - c * (1.0 - n) * pow(t, -n);
    double tn = t - h / dh;
    if (fabs(tn - t) <= 1e-14 * tn) {
      t = tn;
      break;
    }
    t = tn;
  }
#undef HFUN
  if (t < tmin) t = tmin;
  if (t > tmax) t = tmax;
  return t;
}

/* ---------------------------------------------------------------------- */
static int wrapi(int v, int n) { return ((v % n) + n) % n; }

/* Unique node coordinates of the window [lo, hi] on one axis: wrapped on a
 * periodic axis (the whole axis once if the window covers it), clipped
 * otherwise.  Returns the count written to out[]. */
static int axis_window(int lo, int hi, int n, int periodic, int *out) {
  int c = 0;
  if (periodic) {
    if (hi - lo + 1 >= n) {
      for (int v = 0; v < n; ++v) out[c++] = v;
    } else {
      for (int v = lo; v <= hi; ++v) out[c++] = wrapi(v, n);
    }
  } else {
    for (int v = lo; v <= hi; ++v)
      if (v >= 0 && v < n) out[c++] = v;
  }
  return c;
}

/* minimum-image displacement on a periodic axis */
static double min_image(double d, double len, int periodic) {
  if (!periodic) return d;
  return d - len * floor(d / len + 0.5);
}

static int inside_particle(const lbo_sim *s, const lbo_particle *q, int x, int y) {
  double dx = min_image((double)x - q->x, s->nx, s->p.bc_x == LBO_PERIODIC);
  double dy = min_image((double)y - q->y, s->ny, s->p.bc_y == LBO_PERIODIC);
  return dx * dx + dy * dy < q->radius * q->radius;
}

/* Labels of G(t): solid nodes 1; a non-solid node takes 2 + q for the first
 * particle q (index order) whose disc strictly contains it, else 0.  Only
 * nodes in a particle's bounding box can be inside it. */
static void relabel(lbo_sim *s) {
  size_t n = (size_t)s->nx * s->ny;
  for (size_t id = 0; id < n; ++id) s->label[id] = s->solid[id] ? 1 : 0;
  int perx = s->p.bc_x == LBO_PERIODIC, pery = s->p.bc_y == LBO_PERIODIC;
  for (int q = 0; q < s->np; ++q) {
    const lbo_particle *pq = &s->part[q];
    int reach = (int)ceil(pq->radius) + 1;
    int cx = (int)floor(pq->x), cy = (int)floor(pq->y);
    int *xs = (int *)malloc(sizeof(int) * (s->nx + 2 * reach + 2));
    int *ys = (int *)malloc(sizeof(int) * (s->ny + 2 * reach + 2));
    int nxs = axis_window(cx - reach, cx + reach + 1, s->nx, perx, xs);
    int nys = axis_window(cy - reach, cy + reach + 1, s->ny, pery, ys);
    for (int b = 0; b < nys; ++b)
      for (int a = 0; a < nxs; ++a) {
        size_t id = (size_t)ys[b] * s->nx + xs[a];
        if (s->label[id] == 0 && inside_particle(s, pq, xs[a], ys[b])) s->label[id] = (uint8_t)(2 + q);
      }
    free(xs);
    free(ys);
  }
}

lbo_sim *lbo_create(const lbo_params *p, const uint8_t *mask, const double *rho,
                    const double *ux, const double *uy) {
  if (p->nx < 3 || p->ny < 3 || !(p->tau > 0.5)) return NULL;
  if (p->bc_y == LBO_PRESSURE) return NULL;
  if (p->trt && (!(p->magic > 0.0) || p->kT > 0.0)) return NULL;
  lbo_sim *s = (lbo_sim *)calloc(1, sizeof(lbo_sim));
  s->p = *p;
  s->nx = p->nx;
  s->ny = p->ny;
  size_t n = (size_t)p->nx * p->ny;
  s->f = (double *)calloc(9 * n, sizeof(double));
  s->fs = (double *)calloc(9 * n, sizeof(double));
  s->fn = (double *)calloc(9 * n, sizeof(double));
  s->solid = (uint8_t *)calloc(n, 1);
  s->label = (uint8_t *)calloc(n, 1);
  build_basis(s->basis);
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x) {
      size_t id = (size_t)y * s->nx + x;
      int sol = mask ? (mask[id] != 0) : 0;
      if (p->bc_y == LBO_WALL && (y == 0 || y == s->ny - 1)) sol = 1;
      if (p->bc_x == LBO_WALL && (x == 0 || x == s->nx - 1)) sol = 1;
      s->solid[id] = (uint8_t)sol;
      double r = rho ? rho[id] : p->rho0;
      double vx = ux ? ux[id] : 0.0, vy = uy ? uy[id] : 0.0;
      for (int i = 0; i < 9; ++i) s->f[IDX(s, i, x, y)] = sol ? 0.0 : feq(i, r, vx, vy);
    }
  relabel(s);
  return s;
}

void lbo_destroy(lbo_sim *s) {
  if (!s) return;
  free(s->f);
  free(s->fs);
  free(s->fn);
  free(s->solid);
  free(s->label);
  free(s);
}

int lbo_add_particle(lbo_sim *s, const lbo_particle *q) {
  if (s->np >= MAXP - 2 || !(q->radius > 0)) return -1;
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x)
      if (inside_particle(s, q, x, y) && s->label[(size_t)y * s->nx + x] != 0) return -1;
  s->part[s->np] = *q;
  s->part[s->np].fx = s->part[s->np].fy = s->part[s->np].torque = 0.0;
  s->fcu[s->np][0] = s->fcu[s->np][1] = s->fcu[s->np][2] = 0.0;
  s->np += 1;
  relabel(s);
  return 0;
}

/* Is the pull into node (x,y) along direction d a crossing of a particle
 * surface?  Exactly one of the node and its source is inside a particle, both
 * are non-solid, and the outside one is plain fluid.  Returns particle or -1. */
static int crossing(const lbo_sim *s, int lx, int ls) {
  if (lx == 1 || ls == 1) return -1;
  if (lx >= 2 && ls == 0) return lx - 2;
  if (lx == 0 && ls >= 2) return ls - 2;
  return -1;
}

/* velocity of the surface point r_b of particle q: U + Omega z x (r_b - r_c) */
static void surface_velocity(const lbo_sim *s, const lbo_particle *q, double bx, double by,
                             double *vx, double *vy, double *rx, double *ry) {
  *rx = min_image(bx - q->x, s->nx, s->p.bc_x == LBO_PERIODIC);
  *ry = min_image(by - q->y, s->ny, s->p.bc_y == LBO_PERIODIC);
  *vx = q->ux - q->omega * (*ry);
  *vy = q->uy + q->omega * (*rx);
}

/* source coordinate of a pull; returns 0 if it lies outside a non-periodic edge */
static int source_of(const lbo_sim *s, int x, int y, int d, int *sx, int *sy) {
  int a = x - EX[d], b = y - EY[d];
  if (a < 0 || a >= s->nx) {
    if (s->p.bc_x != LBO_PERIODIC) return 0;
    a = wrapi(a, s->nx);
  }
  if (b < 0 || b >= s->ny) {
    if (s->p.bc_y != LBO_PERIODIC) return 0;
    b = wrapi(b, s->ny);
  }
  *sx = a;
  *sy = b;
  return 1;
}

static void collide(lbo_sim *s) {
  const lbo_params *p = &s->p;
  int nx = s->nx, ny = s->ny;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t id = (size_t)y * nx + x;
      if (s->solid[id]) continue;
      double fl[9], rho = 0, jx = 0, jy = 0;
      for (int i = 0; i < 9; ++i) {
        fl[i] = s->f[IDX(s, i, x, y)];
        rho += fl[i];
        jx += fl[i] * EX[i];
        jy += fl[i] * EY[i];
      }
      double tau = p->power_law ? powerlaw_tau(p, fl, rho, jx, jy) : p->tau;
      if (p->trt) {
        /* two relaxation times: the antisymmetric parts, which carry the
         * momentum, relax with 1/tau_m, so the body force shifts u_eq by
         * tau_m g (the momentum input per step stays rho g) */
        const double tm = 0.5 + p->magic / (tau - 0.5);
        const double vx = jx / rho + tm * p->gx, vy = jy / rho + tm * p->gy;
        for (int i = 0; i < 9; ++i) {
          const int o = OPP[i];
          const double fsym = 0.5 * (fl[i] + fl[o]), fanti = 0.5 * (fl[i] - fl[o]);
          const double ei = feq(i, rho, vx, vy), eo = feq(o, rho, vx, vy);
          const double esym = 0.5 * (ei + eo), eanti = 0.5 * (ei - eo);
          s->fs[IDX(s, i, x, y)] = fl[i] - (fsym - esym) / tau - (fanti - eanti) / tm;
        }
        continue;
      }
      double ux = jx / rho + tau * p->gx, uy = jy / rho + tau * p->gy;
      double zeta[9] = {0};
      if (p->kT > 0.0) {
        float th[6];
        lbo_normals(p->seed, p->domain_id, (uint32_t)id, (uint32_t)s->t, th);
        double om = 1.0 / tau;
        double amp = sqrt(rho * p->kT * om * (2.0 - om) / CS2);
        for (int i = 0; i < 9; ++i) {
          double acc = 0.0;
          for (int k = 3; k <= 8; ++k) acc += s->basis[k][i] * (double)th[k - 3];
          zeta[i] = amp * W[i] * acc;
        }
      }
      for (int i = 0; i < 9; ++i)
        s->fs[IDX(s, i, x, y)] = fl[i] - (fl[i] - feq(i, rho, ux, uy)) / tau + zeta[i];
    }
}

/* Link momentum exchange (Eqs. MP1, MP3, MP4).  Eq. MP1 takes the population
 * f' of the exterior node r_v + e_i: the particle is driven by the pulls whose
 * destination is outside it.  The pulls into interior nodes (Eq. MP7) exchange
 * momentum with the interior fluid only; that part is accumulated separately
 * as a diagnostic (fluid momentum changes by minus the sum of both parts). */
static void link_forces(lbo_sim *s) {
  for (int q = 0; q < s->np; ++q) {
    lbo_particle *pq = &s->part[q];
    double F[3] = {0, 0, 0}, Fi[3] = {0, 0, 0};
    int reach = (int)ceil(pq->radius) + 2;
    int cx = (int)floor(pq->x), cy = (int)floor(pq->y);
    int *xs = (int *)malloc(sizeof(int) * (s->nx + 2 * reach + 2));
    int *ys = (int *)malloc(sizeof(int) * (s->ny + 2 * reach + 2));
    int nxs = axis_window(cx - reach, cx + reach + 1, s->nx, s->p.bc_x == LBO_PERIODIC, xs);
    int nys = axis_window(cy - reach, cy + reach + 1, s->ny, s->p.bc_y == LBO_PERIODIC, ys);
    for (int b = 0; b < nys; ++b)
      for (int a = 0; a < nxs; ++a) {
        int x = xs[a], y = ys[b];
        int lx = s->label[(size_t)y * s->nx + x];
        for (int d = 1; d < 9; ++d) {
          int sx, sy;
          if (!source_of(s, x, y, d, &sx, &sy)) continue;
          int ls = s->label[(size_t)sy * s->nx + sx];
          if (crossing(s, lx, ls) != q) continue;
          double bx = x - 0.5 * EX[d], by = y - 0.5 * EY[d];
          double vx, vy, rx, ry;
          surface_velocity(s, pq, bx, by, &vx, &vy, &rx, &ry);
          double ub = vx * EX[d] + vy * EY[d];
          double mag = 2.0 * s->fs[IDX(s, OPP[d], x, y)] + 2.0 * s->p.rho0 * W[d] * ub / CS2;
          double dpx = -EX[d] * mag, dpy = -EY[d] * mag;
          double *acc = lx == 0 ? F : Fi;
          acc[0] += dpx;
          acc[1] += dpy;
          acc[2] += rx * dpy - ry * dpx;
        }
      }
    free(xs);
    free(ys);
    for (int k = 0; k < 3; ++k) {
      s->flink[q][k] = F[k];
      s->flink_int[q][k] = Fi[k];
    }
  }
}

/* LJ-type repulsion (Eq. MP2): along the centre line, magnitude
 * psi (max(gap, floor)/r_it)^-13 for gaps up to r_it; particle-particle uses
 * the surface gap |r_pq| - R_p - R_q, particle-solid the gap |r_s - r_c| - R to
 * every solid node within R + r_it. */
static void lj_forces(lbo_sim *s, double F[][2]) {
  const lbo_params *p = &s->p;
  for (int q = 0; q < s->np; ++q) F[q][0] = F[q][1] = 0.0;
  if (!(p->lj_psi > 0.0)) return;
  int perx = p->bc_x == LBO_PERIODIC, pery = p->bc_y == LBO_PERIODIC;
  for (int a = 0; a < s->np; ++a)
    for (int b = a + 1; b < s->np; ++b) {
      double dx = min_image(s->part[a].x - s->part[b].x, s->nx, perx);
      double dy = min_image(s->part[a].y - s->part[b].y, s->ny, pery);
      double dist = sqrt(dx * dx + dy * dy);
      double gap = dist - s->part[a].radius - s->part[b].radius;
      if (gap > p->lj_rit || dist <= 0.0) continue;
      double g = gap < p->lj_floor ? p->lj_floor : gap;
      double mag = p->lj_psi * pow(g / p->lj_rit, -13.0);
      F[a][0] += mag * dx / dist;
      F[a][1] += mag * dy / dist;
      F[b][0] -= mag * dx / dist;
      F[b][1] -= mag * dy / dist;
    }
  for (int q = 0; q < s->np; ++q) {
    lbo_particle *pq = &s->part[q];
    double lim = pq->radius + p->lj_rit;
    int reach = (int)ceil(lim) + 1;
    int cx = (int)floor(pq->x), cy = (int)floor(pq->y);
    int *xs = (int *)malloc(sizeof(int) * (s->nx + 2 * reach + 2));
    int *ys = (int *)malloc(sizeof(int) * (s->ny + 2 * reach + 2));
    int nxs = axis_window(cx - reach, cx + reach + 1, s->nx, perx, xs);
    int nys = axis_window(cy - reach, cy + reach + 1, s->ny, pery, ys);
    for (int bb = 0; bb < nys; ++bb)
      for (int aa = 0; aa < nxs; ++aa) {
        int x = xs[aa], y = ys[bb];
        if (!s->solid[(size_t)y * s->nx + x]) continue;
        double dx = min_image(pq->x - x, s->nx, perx);
        double dy = min_image(pq->y - y, s->ny, pery);
        double dist = sqrt(dx * dx + dy * dy);
        if (dist > lim || dist <= 0.0) continue;
        double gap = dist - pq->radius;
        double g = gap < p->lj_floor ? p->lj_floor : gap;
        double mag = p->lj_psi * pow(g / p->lj_rit, -13.0);
        F[q][0] += mag * dx / dist;
        F[q][1] += mag * dy / dist;
      }
    free(xs);
    free(ys);
  }
}

static void stream(lbo_sim *s) {
  int nx = s->nx, ny = s->ny;
  double rho0 = s->p.rho0;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t id = (size_t)y * nx + x;
      if (s->solid[id]) {
        for (int d = 0; d < 9; ++d) s->fn[IDX(s, d, x, y)] = 0.0;
        continue;
      }
      int lx = s->label[id];
      s->fn[IDX(s, 0, x, y)] = s->fs[IDX(s, 0, x, y)];
      for (int d = 1; d < 9; ++d) {
        int sx, sy;
        if (!source_of(s, x, y, d, &sx, &sy)) {
          s->fn[IDX(s, d, x, y)] = NAN; /* unknown: filled by the pressure rule */
          continue;
        }
        int ls = s->label[(size_t)sy * nx + sx];
        double v;
        if (ls == 1) {
          v = s->fs[IDX(s, OPP[d], x, y)]; /* stationary halfway bounce-back */
        } else {
          int q = crossing(s, lx, ls);
          if (q >= 0) {
            /* moving-wall bounce-back, Eqs. MP7 (interior) / MP8 (exterior) */
            double vx, vy, rx, ry;
            surface_velocity(s, &s->part[q], x - 0.5 * EX[d], y - 0.5 * EY[d], &vx, &vy,
                             &rx, &ry);
            double ub = vx * EX[d] + vy * EY[d];
            v = s->fs[IDX(s, OPP[d], x, y)] + 2.0 * rho0 * W[d] * ub / CS2;
          } else {
            v = s->fs[IDX(s, d, sx, sy)];
          }
        }
        s->fn[IDX(s, d, x, y)] = v;
      }
    }
}

/* Zou & He (1997) density boundary on the x faces, zero transverse velocity. */
static void pressure_faces(lbo_sim *s) {
  if (s->p.bc_x != LBO_PRESSURE) return;
  int nx = s->nx;
  for (int y = 0; y < s->ny; ++y) {
    size_t id = (size_t)y * nx;
    if (!s->solid[id]) {
      double f[9];
      for (int i = 0; i < 9; ++i) f[i] = s->fn[IDX(s, i, 0, y)];
      double r = s->p.rho_in;
      double ux = 1.0 - (f[0] + f[2] + f[4] + 2.0 * (f[3] + f[6] + f[7])) / r;
      s->fn[IDX(s, 1, 0, y)] = f[3] + (2.0 / 3.0) * r * ux;
      s->fn[IDX(s, 5, 0, y)] = f[7] - 0.5 * (f[2] - f[4]) + (1.0 / 6.0) * r * ux;
      s->fn[IDX(s, 8, 0, y)] = f[6] + 0.5 * (f[2] - f[4]) + (1.0 / 6.0) * r * ux;
    }
    id = (size_t)y * nx + (nx - 1);
    if (!s->solid[id]) {
      double f[9];
      for (int i = 0; i < 9; ++i) f[i] = s->fn[IDX(s, i, nx - 1, y)];
      double r = s->p.rho_out;
      double ux = -1.0 + (f[0] + f[2] + f[4] + 2.0 * (f[1] + f[5] + f[8])) / r;
      s->fn[IDX(s, 3, nx - 1, y)] = f[1] - (2.0 / 3.0) * r * ux;
      s->fn[IDX(s, 7, nx - 1, y)] = f[5] + 0.5 * (f[2] - f[4]) - (1.0 / 6.0) * r * ux;
      s->fn[IDX(s, 6, nx - 1, y)] = f[8] - 0.5 * (f[2] - f[4]) - (1.0 / 6.0) * r * ux;
    }
  }
}

static void node_moments(const lbo_sim *s, const double *f, int x, int y, double *rho,
                         double *ux, double *uy) {
  double r = 0, jx = 0, jy = 0;
  for (int i = 0; i < 9; ++i) {
    double v = f[IDX(s, i, x, y)];
    r += v;
    jx += v * EX[i];
    jy += v * EY[i];
  }
  *rho = r;
  *ux = jx / r + 0.5 * s->p.gx;
  *uy = jy / r + 0.5 * s->p.gy;
}

/* Newton-Euler (Eqs. MP5, MP6) with m = rho_p pi R^2, I = m R^2 / 2, then
 * relabelling and the covered/uncovered node terms for the next step.  With
 * force_average the velocity update takes the mean of this step's and the
 * previous step's total force and torque (the previous ones are the
 * particle's fx, fy, torque before they are overwritten here): an optional
 * stabilisation of the explicit update, not part of Eqs. MP5-MP6. */
static void move_particles(lbo_sim *s, double lj[][2]) {
  const lbo_params *p = &s->p;
  int perx = p->bc_x == LBO_PERIODIC, pery = p->bc_y == LBO_PERIODIC;
  for (int q = 0; q < s->np; ++q) {
    lbo_particle *pq = &s->part[q];
    double Fx = s->flink[q][0] + s->fcu[q][0] + lj[q][0];
    double Fy = s->flink[q][1] + s->fcu[q][1] + lj[q][1];
    double T = s->flink[q][2] + s->fcu[q][2];
    double Fxu = Fx, Fyu = Fy, Tu = T;
    if (p->force_average) {
      Fxu = 0.5 * (Fx + pq->fx);
      Fyu = 0.5 * (Fy + pq->fy);
      Tu = 0.5 * (T + pq->torque);
    }
    pq->fx = Fx;
    pq->fy = Fy;
    pq->torque = T;
    if (pq->flags & LBO_PARTICLE_FIXED) continue;
    double rhop = pq->density_ratio * p->rho0;
    double m = rhop * M_PI * pq->radius * pq->radius;
    double I = 0.5 * m * pq->radius * pq->radius;
    double ux0 = pq->ux, uy0 = pq->uy;
    pq->ux = ux0 + Fxu / m + (1.0 - p->rho0 / rhop) * p->gx;
    pq->uy = uy0 + Fyu / m + (1.0 - p->rho0 / rhop) * p->gy;
    pq->omega = pq->omega + Tu / I;
    pq->x += ux0;
    pq->y += uy0;
    if (perx) {
      if (pq->x >= s->nx) pq->x -= s->nx;
      if (pq->x < 0) pq->x += s->nx;
    }
    if (pery) {
      if (pq->y >= s->ny) pq->y -= s->ny;
      if (pq->y < 0) pq->y += s->ny;
    }
  }
  size_t n = (size_t)s->nx * s->ny;
  uint8_t *old = (uint8_t *)malloc(n);
  memcpy(old, s->label, n);
  relabel(s);
  for (int q = 0; q < s->np; ++q) s->fcu[q][0] = s->fcu[q][1] = s->fcu[q][2] = 0.0;
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x) {
      size_t id = (size_t)y * s->nx + x;
      int a = old[id], b = s->label[id];
      if (a == b) continue;
      double rho, ux, uy;
      node_moments(s, s->f, x, y, &rho, &ux, &uy);
      for (int side = 0; side < 2; ++side) {
        int lab = side == 0 ? a : b;
        if (lab < 2) continue;
        int q = lab - 2;
        double sign = side == 0 ? -1.0 : 1.0; /* uncovered : covered */
        lbo_particle *pq = &s->part[q];
        double fx = sign * rho * (ux - pq->ux), fy = sign * rho * (uy - pq->uy);
        double rx = min_image(x - pq->x, s->nx, perx), ry = min_image(y - pq->y, s->ny, pery);
        s->fcu[q][0] += fx;
        s->fcu[q][1] += fy;
        s->fcu[q][2] += rx * fy - ry * fx;
      }
    }
  free(old);
}

static void step(lbo_sim *s) {
  double lj[MAXP][2];
  collide(s);
  if (s->np > 0) {
    link_forces(s);
    lj_forces(s, lj);
  }
  stream(s);
  pressure_faces(s);
  double *tmp = s->f;
  s->f = s->fn;
  s->fn = tmp;
  if (s->np > 0) move_particles(s, lj);
  s->t += 1;
}

void lbo_run(lbo_sim *s, int64_t nsteps) {
  for (int64_t k = 0; k < nsteps; ++k) step(s);
}

int64_t lbo_time(const lbo_sim *s) { return s->t; }

void lbo_moments(const lbo_sim *s, double *rho, double *ux, double *uy) {
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x) {
      size_t id = (size_t)y * s->nx + x;
      if (s->solid[id]) {
        rho[id] = ux[id] = uy[id] = 0.0;
        continue;
      }
      node_moments(s, s->f, x, y, &rho[id], &ux[id], &uy[id]);
    }
}

void lbo_populations(const lbo_sim *s, double *f) {
  memcpy(f, s->f, 9 * (size_t)s->nx * s->ny * sizeof(double));
}

void lbo_set_populations(lbo_sim *s, const double *f) {
  memcpy(s->f, f, 9 * (size_t)s->nx * s->ny * sizeof(double));
}

void lbo_labels(const lbo_sim *s, uint8_t *out) {
  memcpy(out, s->label, (size_t)s->nx * s->ny);
}

int lbo_num_particles(const lbo_sim *s) { return s->np; }

void lbo_get_particles(const lbo_sim *s, lbo_particle *out) {
  memcpy(out, s->part, (size_t)s->np * sizeof(lbo_particle));
}

double lbo_mass(const lbo_sim *s) {
  double m = 0.0;
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x) {
      if (s->solid[(size_t)y * s->nx + x]) continue;
      for (int i = 0; i < 9; ++i) m += s->f[IDX(s, i, x, y)];
    }
  return m;
}

void lbo_momentum(const lbo_sim *s, double *jx, double *jy) {
  double ax = 0.0, ay = 0.0;
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x) {
      if (s->solid[(size_t)y * s->nx + x]) continue;
      for (int i = 0; i < 9; ++i) {
        ax += s->f[IDX(s, i, x, y)] * EX[i];
        ay += s->f[IDX(s, i, x, y)] * EY[i];
      }
    }
  *jx = ax;
  *jy = ay;
}

void lbo_link_forces(const lbo_sim *s, double *out) {
  for (int q = 0; q < s->np; ++q)
    for (int k = 0; k < 3; ++k) {
      out[6 * q + k] = s->flink[q][k];
      out[6 * q + 3 + k] = s->flink_int[q][k];
    }
}
