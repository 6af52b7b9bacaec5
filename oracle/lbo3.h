/*
 * lbo3.h -- CPU oracle (FP64) of the three-dimensional lattice-Boltzmann step
 * on D3Q19 or D3Q27: BGK with the velocity-shift body force (Sec. 2), or its
 * two-relaxation-time (TRT) variant, optionally with thermal noise,
 * pull streaming with periodic wrap, halfway bounce-back on solid nodes.
 * TEST INFRASTRUCTURE ONLY.
 *
 * Arrays: nodes [nz][ny][nx] (x fastest), populations [q][nz][ny][nx].
 * Step order: collide every fluid node, then pull-stream.  The reported
 * velocity is u = j/rho + g/2.
 */
#ifndef LBO3_H
#define LBO3_H

#include <stddef.h>
#include <stdint.h>

typedef struct {
  int32_t nx, ny, nz;
  int32_t wall_x, wall_y, wall_z; /* nonzero: the outermost planes are solid */
  double tau, rho0, gx, gy, gz;
  /* trt nonzero: the symmetric part of each population pair relaxes with
   * 1/tau, the antisymmetric part with 1/tau_minus, where
   * (tau - 1/2)(tau_minus - 1/2) = magic */
  int32_t trt;
  double magic;
  int32_t q; /* 19 (D3Q19) or 27 (D3Q27) */
  /* power_law nonzero: local tau* of the power-law fluid (Sec. 5) from the
   * non-equilibrium stress, flow index n_index, consistency K, clamped to
   * [tau_min, tau_max]; tau is then unused (TRT takes tau_minus from tau*) */
  int32_t power_law;
  double n_index, K, tau_min, tau_max;
  /* kT > 0: thermal noise of the fluctuating method (Sec. 4) added to every
   * collision (with TRT, each of the symmetric and antisymmetric parts at
   * its own rate's amplitude); Philox key (lo32(seed), hi32(seed)) */
  double kT;
  uint64_t seed;
} lbo3_params;

typedef struct lbo3_sim lbo3_sim;

lbo3_sim *lbo3_create(const lbo3_params *p, const uint8_t *mask, const double *rho,
                      const double *ux, const double *uy, const double *uz);
void lbo3_destroy(lbo3_sim *s);
void lbo3_run(lbo3_sim *s, int64_t nsteps);
int64_t lbo3_time(const lbo3_sim *s);
void lbo3_moments(const lbo3_sim *s, double *rho, double *ux, double *uy, double *uz);
void lbo3_populations(const lbo3_sim *s, double *f);
double lbo3_mass(const lbo3_sim *s);
void lbo3_momentum(const lbo3_sim *s, double *j);
/* the velocity set and weights of the q-velocity lattice (q = 19 or 27) */
void lbo3_lattice(int q, int *ex, int *ey, int *ez, double *w);

#endif
