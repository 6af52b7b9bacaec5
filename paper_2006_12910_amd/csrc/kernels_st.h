// kernels_st.h -- instantiates the kernels of one storage format (LBK_ST) and
// exposes them through a KernelSet.  Included once per kern_*.hip file so the
// formats compile in parallel.
#pragma once

#include "aux_impl.h"
#include "launch.h"
#include "particles_impl.h"
#include "sweep2_impl.h"
#include "sweep_impl.h"

namespace lbk {
namespace {

constexpr int ST = LBK_ST;

template <int FEAT, int PLM, int WIDE>
void sweep_l(const DevDomain *doms, const int *prefix, int ndom, int kstep, int blocks, int part,
             hipStream_t s) {
  hipLaunchKernelGGL((k_sweep<ST, FEAT, PLM, WIDE>), dim3(blocks), dim3(256), 0, s, doms, prefix,
                     ndom, kstep, part);
}
template <int FEAT, int PLM>
void sweep2_l(const DevDomain *doms, const int *prefix2, int ndom, int kstep, int which, int blocks,
              int rows, hipStream_t s) {
  constexpr int H0 = two_step_rows_of(ST, 0), H1 = two_step_rows_of(ST, 1),
                H2 = two_step_rows_of(ST, 2);
  if (rows == H0)
    hipLaunchKernelGGL((k_sweep2<ST, FEAT, H0, PLM>), dim3(blocks), dim3(256), 0, s, doms, prefix2,
                       ndom, kstep, which);
  else if (rows == H2)
    hipLaunchKernelGGL((k_sweep2<ST, FEAT, H2, PLM>), dim3(blocks), dim3(256), 0, s, doms, prefix2,
                       ndom, kstep, which);
  else
    hipLaunchKernelGGL((k_sweep2<ST, FEAT, H1, PLM>), dim3(blocks), dim3(256), 0, s, doms, prefix2,
                       ndom, kstep, which);
}
template <int FEAT, int PLM, int WIDE>
void init_l(const DevDomain *dom, const double *rho, const double *ux, const double *uy, int row0,
            int nrows, int pitch, hipStream_t s) {
  const long long n = (long long)nrows * pitch;
  hipLaunchKernelGGL((k_init<ST, FEAT, PLM, WIDE>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     dom, rho, ux, uy, row0, nrows);
}
void pre_l(const DevDomain *doms, const PItem *items, int nitems, int kstep, hipStream_t s) {
  hipLaunchKernelGGL((k_pre<ST>), dim3(nitems), dim3(256), 0, s, doms, items, kstep);
}
void post_l(const DevDomain *doms, const PItem *items, int nitems, int kstep, hipStream_t s) {
  hipLaunchKernelGGL((k_post<ST>), dim3(nitems), dim3(256), 0, s, doms, items, kstep);
}
void post_pre_l(const DevDomain *doms, const PItem *items, int nitems, int kstep, hipStream_t s) {
  hipLaunchKernelGGL((k_post_pre<ST>), dim3(nitems), dim3(256), 0, s, doms, items, kstep);
}
void mass_l(const DevDomain *doms, const int *prefix, int ndom, int blocks, double *alt,
            hipStream_t s) {
  hipLaunchKernelGGL((k_mass_partial<ST>), dim3(blocks), dim3(256), 0, s, doms, prefix, ndom, alt);
}
void moments_l(const DevDomain *dom, double *rho, double *ux, double *uy, int row0, int nrows,
               int nx, hipStream_t s) {
  const long long n = (long long)nrows * nx;
  hipLaunchKernelGGL((k_moments<ST>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dom,
                     rho, ux, uy, row0, nrows);
}
void export_l(const DevDomain *dom, double *out, int row0, int nrows, int nx, hipStream_t s) {
  const long long n = (long long)nrows * nx;
  hipLaunchKernelGGL((k_export<ST>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dom, out,
                     row0, nrows);
}
void import_l(const DevDomain *dom, const double *in, int row0, int nrows, int nx,
              hipStream_t s) {
  const long long n = (long long)nrows * nx;
  hipLaunchKernelGGL((k_import<ST>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dom, in,
                     row0, nrows);
}

void mirror_l(const DevDomain *dom, int nx, int ny, hipStream_t s) {
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL((k_mirror<ST>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dom);
}

template <int FEAT, int PLM, int WIDE> void fill(KernelSet *k) {
  k->sweep = sweep_l<FEAT, PLM, WIDE>;
  // the two-step sweep: plain and obstacle (label) sweeps, and the power-law
  // sweep of label domains (walls as solid label rows); not with noise
  if constexpr ((FEAT & F_NOISE) == 0 && WIDE == 0 &&
                ((FEAT & F_POWER) == 0 || (FEAT & F_LABELS) != 0))
    k->sweep2 = sweep2_l<FEAT, PLM>;
  else
    k->sweep2 = nullptr;
  k->init = init_l<FEAT, PLM, WIDE>;
  k->pre = pre_l;
  k->post = post_l;
  k->post_pre = post_pre_l;
  k->mass_partial = mass_l;
  k->moments = moments_l;
  k->export_f = export_l;
  k->import_f = import_l;
  k->mirror = mirror_l;
}

template <int BASE, int WIDE> bool pick_power(int feat, int plm, KernelSet *k) {
  if (!(feat & F_POWER)) { fill<BASE, PL_GENERIC, WIDE>(k); return true; }
  switch (plm) {
    case PL_GENERIC: fill<BASE | F_POWER, PL_GENERIC, WIDE>(k); return true;
    case PL_HALF: fill<BASE | F_POWER, PL_HALF, WIDE>(k); return true;
    case PL_3Q: fill<BASE | F_POWER, PL_3Q, WIDE>(k); return true;
    case PL_3H: fill<BASE | F_POWER, PL_3H, WIDE>(k); return true;
  }
  return false;
}

template <int WIDE> bool pick(int feat, int plm, KernelSet *k) {
  switch (feat & (F_LABELS | F_NOISE | F_TRT)) {
    case 0: return pick_power<0, WIDE>(feat, plm, k);
    case F_LABELS: return pick_power<F_LABELS, WIDE>(feat, plm, k);
    case F_NOISE: return pick_power<F_NOISE, WIDE>(feat, plm, k);
    case F_LABELS | F_NOISE: return pick_power<F_LABELS | F_NOISE, WIDE>(feat, plm, k);
    case F_TRT: return pick_power<F_TRT, WIDE>(feat, plm, k);
    case F_LABELS | F_TRT: return pick_power<F_LABELS | F_TRT, WIDE>(feat, plm, k);
  }
  return false;  // TRT with noise is refused at validation
}

}  // namespace

bool LBK_GETTER(int feat, int plm, int wide, KernelSet *k) {
  if (ST == ST_F64 || !wide) return pick<0>(feat, plm, k);
  return pick<1>(feat, plm, k);
}

}  // namespace lbk
