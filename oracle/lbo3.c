/*
 * lbo3.c -- CPU oracle (FP64) of the three-dimensional D3Q19 and D3Q27
 * variants of the lattice-Boltzmann step (the 3D lattices the paper names as
 * its next step, Sec. 8): BGK collision with the velocity-shift body force of
 * Sec. 2
 * (u_eq = j/rho + tau g), pull streaming, halfway bounce-back on solid
 * nodes.  Optionally the two-relaxation-time (TRT) collision: populations
 * split into parts symmetric and antisymmetric under e -> -e, relaxed with
 * rates 1/tau and 1/tau_minus, (tau - 1/2)(tau_minus - 1/2) = magic; the
 * body force then shifts u_eq by tau_minus g, since the antisymmetric part
 * carries the momentum (reading stated in the design notes: the paper uses
 * BGK only).  Optionally thermal noise (Sec. 4) in the form stated at
 * noise3() below.  TEST INFRASTRUCTURE ONLY: used by the tests and the
 * benchmark's CPU-baseline leg, never by the library.
 *
 * Plain on purpose: full populations f (not deviations), two arrays, one
 * loop per step of the method.  Build flags: -O2 -fno-fast-math
 * -ffp-contract=off.
 */
#include "lbo3.h"

#include "lbo.h" /* the Philox / Box-Muller normals of the D2Q9 oracle */

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* The rest velocity, the six axis velocities, the twelve edge velocities (two
 * unit components) and, for D3Q27 only, the eight corner velocities (three
 * unit components); opposite velocities sit at (i, i + 1) for odd i.
 * D3Q19 weights 1/3, 1/18, 1/36; D3Q27 weights the products of the
 * one-dimensional three-velocity weights 2/3 (component 0) and 1/6
 * (component +-1): 8/27, 2/27, 1/54, 1/216.  c_s^2 = 1/3 on both. */
static const int EX[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                           1, -1, 1, -1, 1, -1, -1, 1};
static const int EY[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                           1, -1, 1, -1, -1, 1, 1, -1};
static const int EZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                           1, -1, -1, 1, 1, -1, 1, -1};

static double w1d(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
static double weight(int q, int i) {
  if (q == 27) return w1d(EX[i]) * w1d(EY[i]) * w1d(EZ[i]);
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
static int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

struct lbo3_sim {
  lbo3_params p;
  int64_t t;
  int q;
  double w[27];
  double *f, *fs; /* pre-collision f(t) and post-collision f*(t), [q][nz][ny][nx] */
  uint8_t *solid; /* [nz][ny][nx] */
};

#define NODE(s, x, y, z) (((size_t)(z) * (s)->p.ny + (y)) * (s)->p.nx + (x))
#define IDX(s, i, x, y, z) ((size_t)(i) * (size_t)(s)->p.nx * (s)->p.ny * (s)->p.nz + NODE(s, x, y, z))

void lbo3_lattice(int q, int *ex, int *ey, int *ez, double *w) {
  for (int i = 0; i < q; ++i) {
    ex[i] = EX[i];
    ey[i] = EY[i];
    ez[i] = EZ[i];
    w[i] = weight(q, i);
  }
}

/* Equilibrium of Eq. LB2 (c_s^2 = 1/3) with weight w. */
static double feq(int i, double w, double rho, double ux, double uy, double uz) {
  double eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
  double uu = ux * ux + uy * uy + uz * uz;
  return w * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

lbo3_sim *lbo3_create(const lbo3_params *p, const uint8_t *mask, const double *rho,
                      const double *ux, const double *uy, const double *uz) {
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) return NULL;
  if (!p->power_law && !(p->tau > 0.5)) return NULL;
  if (p->power_law && (!(p->tau_min > 0.5) || !(p->tau_max >= p->tau_min) || !(p->n_index > 0.0) ||
                       !(p->K > 0.0)))
    return NULL;
  if (p->trt && !(p->magic > 0.0)) return NULL;
  if (p->q != 19 && p->q != 27) return NULL;
  if (!(p->kT >= 0.0)) return NULL;
  if (p->kT > 0.0 && (double)p->nx * p->ny * p->nz > 4294967295.0) return NULL;
  lbo3_sim *s = (lbo3_sim *)calloc(1, sizeof(lbo3_sim));
  s->p = *p;
  s->q = p->q;
  for (int i = 0; i < s->q; ++i) s->w[i] = weight(s->q, i);
  size_t n = (size_t)p->nx * p->ny * p->nz;
  s->f = (double *)calloc((size_t)s->q * n, sizeof(double));
  s->fs = (double *)calloc((size_t)s->q * n, sizeof(double));
  s->solid = (uint8_t *)calloc(n, 1);
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        size_t id = NODE(s, x, y, z);
        int sol = mask ? (mask[id] != 0) : 0;
        if (p->wall_x && (x == 0 || x == p->nx - 1)) sol = 1;
        if (p->wall_y && (y == 0 || y == p->ny - 1)) sol = 1;
        if (p->wall_z && (z == 0 || z == p->nz - 1)) sol = 1;
        s->solid[id] = (uint8_t)sol;
        double r = rho ? rho[id] : p->rho0;
        double vx = ux ? ux[id] : 0.0, vy = uy ? uy[id] : 0.0, vz = uz ? uz[id] : 0.0;
        for (int i = 0; i < s->q; ++i)
          s->f[IDX(s, i, x, y, z)] = sol ? 0.0 : feq(i, s->w[i], r, vx, vy, vz);
      }
  return s;
}

void lbo3_destroy(lbo3_sim *s) {
  if (!s) return;
  free(s->f);
  free(s->fs);
  free(s->solid);
  free(s);
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* relaxation time of the antisymmetric parts: tau itself for BGK, else the
 * one that makes (tau - 1/2)(tau_minus - 1/2) = magic */
static double tau_minus(const lbo3_params *p, double tau) {
  return p->trt ? 0.5 + p->magic / (tau - 0.5) : tau;
}

/* Power-law relaxation time (Sec. 5) on the 3D lattice, the 2D oracle's
 * reading with the full stress tensor: Pi = sum e e (f - feq(rho, j/rho +
 * g/2)), A = 3 |Pi|_F / (sqrt(2) rho) (|Pi|_F over all nine components),
 * gamma_dot = A / tau, nu* = K gamma_dot^(n-1), tau* = 1/2 + 3 nu*: tau*
 * is the root of h(tau) = tau - 1/2 - 3 K A^(n-1) tau^(1-n), found by
 * Newton from the bracket end on the side where h keeps its curvature, then
 * clamped to [tau_min, tau_max]. */
static double powerlaw_tau3(const lbo3_sim *s, const double *fl, double rho, double jx, double jy,
                            double jz) {
  const lbo3_params *p = &s->p;
  double n = p->n_index, xi = p->K;
  if (n == 1.0) {
    double t = 0.5 + 3.0 * xi;
    return t < p->tau_min ? p->tau_min : (t > p->tau_max ? p->tau_max : t);
  }
  double ux = jx / rho + 0.5 * p->gx, uy = jy / rho + 0.5 * p->gy, uz = jz / rho + 0.5 * p->gz;
  double pi[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int i = 0; i < s->q; ++i) {
    double d = fl[i] - feq(i, s->w[i], rho, ux, uy, uz);
    int e[3] = {EX[i], EY[i], EZ[i]};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) pi[a][b] += e[a] * e[b] * d;
  }
  double fro2 = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) fro2 += pi[a][b] * pi[a][b];
  double A = 3.0 * sqrt(fro2) / (sqrt(2.0) * rho);
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

/* Thermal noise of one collision (Sec. 4, Eqs. NP1-NP2 carried to 3D).  The
 * D2Q9 method puts independent unit normals Theta_k on each non-conserved
 * mode of a basis orthonormal under sum_i w_i chi_ki chi_li, scaled by
 * sqrt(rho kT omega (2 - omega) / c_s^2) and mapped back with w_i; the noise
 * then has covariance amp^2 (W - w w^T - 3 (W e)(W e)^T), W = diag(w), the
 * part of W with the mass and momentum modes removed.  The same Gaussian is
 * drawn here without a basis: q independent unit normals xi_i, eta_i =
 * sqrt(w_i) xi_i (covariance W), minus their mass and momentum parts,
 * zeta_i = amp (eta_i - w_i S - 3 w_i e_i.V), S = sum eta, V = sum e eta.
 * The xi come from Philox blocks 0, 1, ... of (node, step): block b gives
 * xi_{6b} .. xi_{6b+5}, the first q are used.
 * With TRT the parts of eta symmetric and antisymmetric under e -> -e relax
 * with omega = 1/tau and 1/tau_minus; each gets its own amplitude, mass
 * leaving the symmetric part and momentum the antisymmetric one:
 * zeta = amp+ (eta_s - w S) + amp- (eta_a - 3 w e.V), the two parts being
 * orthogonal in the weights (BGK: amp+ = amp-, the form above). */
static void noise3(const lbo3_sim *s, uint32_t node, double rho, double tau, double tau_m,
                   double *zeta) {
  const lbo3_params *p = &s->p;
  const int q = s->q;
  float xi[30];
  for (int b = 0; 6 * b < q; ++b)
    lbo_normals_block(p->seed, 0u, node, (uint32_t)s->t, (uint32_t)b, xi + 6 * b);
  const double om = 1.0 / tau, omm = 1.0 / tau_m;
  const double amp = sqrt(rho * p->kT * om * (2.0 - om) * 3.0);     /* 1 / c_s^2 = 3 */
  const double ampm = sqrt(rho * p->kT * omm * (2.0 - omm) * 3.0);
  double eta[27], S = 0.0, V[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < q; ++i) {
    eta[i] = sqrt(s->w[i]) * (double)xi[i];
    S += eta[i];
    V[0] += EX[i] * eta[i];
    V[1] += EY[i] * eta[i];
    V[2] += EZ[i] * eta[i];
  }
  for (int i = 0; i < q; ++i) {
    const int o = opposite(i);
    const double es = 0.5 * (eta[i] + eta[o]), ea = 0.5 * (eta[i] - eta[o]);
    const double eV = EX[i] * V[0] + EY[i] * V[1] + EZ[i] * V[2];
    zeta[i] = amp * (es - s->w[i] * S) + ampm * (ea - 3.0 * s->w[i] * eV);
  }
}

/* collide every fluid node into fs */
static void collide(lbo3_sim *s) {
  const lbo3_params *p = &s->p;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        if (s->solid[NODE(s, x, y, z)]) continue;
        double fl[27], rho = 0, jx = 0, jy = 0, jz = 0;
        for (int i = 0; i < s->q; ++i) {
          fl[i] = s->f[IDX(s, i, x, y, z)];
          rho += fl[i];
          jx += fl[i] * EX[i];
          jy += fl[i] * EY[i];
          jz += fl[i] * EZ[i];
        }
        const double tau = p->power_law ? powerlaw_tau3(s, fl, rho, jx, jy, jz) : p->tau;
        const double tm = tau_minus(p, tau);
        double ux = jx / rho + tm * p->gx;
        double uy = jy / rho + tm * p->gy;
        double uz = jz / rho + tm * p->gz;
        if (!p->trt) {
          double zeta[27] = {0.0};
          if (p->kT > 0.0) noise3(s, (uint32_t)NODE(s, x, y, z), rho, tau, tau, zeta);
          for (int i = 0; i < s->q; ++i)
            s->fs[IDX(s, i, x, y, z)] =
                fl[i] - (fl[i] - feq(i, s->w[i], rho, ux, uy, uz)) / tau + zeta[i];
          continue;
        }
        double zeta[27] = {0.0};
        if (p->kT > 0.0) noise3(s, (uint32_t)NODE(s, x, y, z), rho, tau, tm, zeta);
        for (int i = 0; i < s->q; ++i) {
          const int o = opposite(i);
          const double fsym = 0.5 * (fl[i] + fl[o]), fanti = 0.5 * (fl[i] - fl[o]);
          const double ei = feq(i, s->w[i], rho, ux, uy, uz), eo = feq(o, s->w[o], rho, ux, uy, uz);
          const double esym = 0.5 * (ei + eo), eanti = 0.5 * (ei - eo);
          s->fs[IDX(s, i, x, y, z)] = fl[i] - (fsym - esym) / tau - (fanti - eanti) / tm + zeta[i];
        }
      }
}

/* pull: f_i(x, t+1) = f*_i(x - e_i) with periodic wrap; halfway bounce-back
 * f*_{opp i}(x) where the source is solid */
static void stream(lbo3_sim *s) {
  const lbo3_params *p = &s->p;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        if (s->solid[NODE(s, x, y, z)]) {
          for (int i = 0; i < s->q; ++i) s->f[IDX(s, i, x, y, z)] = 0.0;
          continue;
        }
        for (int i = 0; i < s->q; ++i) {
          int sx = wrap(x - EX[i], p->nx), sy = wrap(y - EY[i], p->ny), sz = wrap(z - EZ[i], p->nz);
          s->f[IDX(s, i, x, y, z)] = s->solid[NODE(s, sx, sy, sz)]
                                         ? s->fs[IDX(s, opposite(i), x, y, z)]
                                         : s->fs[IDX(s, i, sx, sy, sz)];
        }
      }
}

void lbo3_run(lbo3_sim *s, int64_t nsteps) {
  for (int64_t k = 0; k < nsteps; ++k) {
    collide(s);
    stream(s);
    s->t += 1;
  }
}

int64_t lbo3_time(const lbo3_sim *s) { return s->t; }

void lbo3_moments(const lbo3_sim *s, double *rho, double *ux, double *uy, double *uz) {
  const lbo3_params *p = &s->p;
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        size_t id = NODE(s, x, y, z);
        if (s->solid[id]) {
          rho[id] = ux[id] = uy[id] = uz[id] = 0.0;
          continue;
        }
        double r = 0, jx = 0, jy = 0, jz = 0;
        for (int i = 0; i < s->q; ++i) {
          double v = s->f[IDX(s, i, x, y, z)];
          r += v;
          jx += v * EX[i];
          jy += v * EY[i];
          jz += v * EZ[i];
        }
        rho[id] = r;
        ux[id] = jx / r + 0.5 * p->gx;
        uy[id] = jy / r + 0.5 * p->gy;
        uz[id] = jz / r + 0.5 * p->gz;
      }
}

void lbo3_populations(const lbo3_sim *s, double *f) {
  memcpy(f, s->f, (size_t)s->q * s->p.nx * s->p.ny * s->p.nz * sizeof(double));
}

double lbo3_mass(const lbo3_sim *s) {
  const lbo3_params *p = &s->p;
  double m = 0.0;
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        if (s->solid[NODE(s, x, y, z)]) continue;
        for (int i = 0; i < s->q; ++i) m += s->f[IDX(s, i, x, y, z)];
      }
  return m;
}

void lbo3_momentum(const lbo3_sim *s, double *j) {
  const lbo3_params *p = &s->p;
  double a[3] = {0, 0, 0};
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        if (s->solid[NODE(s, x, y, z)]) continue;
        for (int i = 0; i < s->q; ++i) {
          double v = s->f[IDX(s, i, x, y, z)];
          a[0] += v * EX[i];
          a[1] += v * EY[i];
          a[2] += v * EZ[i];
        }
      }
  j[0] = a[0];
  j[1] = a[1];
  j[2] = a[2];
}
