// launch.h -- host-side entry points into the kernels (internal to the library).
#pragma once

#include "lb_device.h"

namespace lbk {

struct KernelSet {
  // part: 0 every tile; 1 / 2 the tiles outside / inside the particle
  // coupling's reach (near_tiles of the step)
  void (*sweep)(const DevDomain *doms, const int *prefix, int ndom, int kstep, int blocks, int part,
                hipStream_t s);
  // two steps per launch (periodic plain/obstacle domains), tiles of `rows`
  // output rows (one of two_step_rows_of); null where the feature set has no
  // two-step kernel
  void (*sweep2)(const DevDomain *doms, const int *prefix2, int ndom, int kstep, int which,
                 int blocks, int rows, hipStream_t s);
  void (*init)(const DevDomain *dom, const double *rho, const double *ux, const double *uy,
               int row0, int nrows, int pitch, hipStream_t s);
  // particle coupling before and after the sweep (one workgroup per particle)
  void (*pre)(const DevDomain *doms, const PItem *items, int nitems, int kstep, hipStream_t s);
  void (*post)(const DevDomain *doms, const PItem *items, int nitems, int kstep, hipStream_t s);
  // post of step kstep and pre of step kstep + 1 in one launch (launches in
  // which no domain holds more than one particle)
  void (*post_pre)(const DevDomain *doms, const PItem *items, int nitems, int kstep,
                   hipStream_t s);
  // FP64 density partial sums of ndom domains (mass block prefix per domain),
  // into each domain's partials, or into alt (one domain)
  void (*mass_partial)(const DevDomain *doms, const int *prefix, int ndom, int blocks,
                       double *alt, hipStream_t s);
  void (*moments)(const DevDomain *dom, double *rho, double *ux, double *uy, int row0, int nrows,
                  int nx, hipStream_t s);
  void (*export_f)(const DevDomain *dom, double *out, int row0, int nrows, int nx, hipStream_t s);
  void (*import_f)(const DevDomain *dom, const double *in, int row0, int nrows, int nx,
                   hipStream_t s);
  void (*mirror)(const DevDomain *dom, int nx, int ny, hipStream_t s);
};

// Kernel set of a storage format / feature set / power-law specialisation /
// arithmetic width (wide = FP64 arithmetic with any storage).
bool kernels_f64(int feat, int plm, int wide, KernelSet *k);
bool kernels_f32(int feat, int plm, int wide, KernelSet *k);
bool kernels_f16(int feat, int plm, int wide, KernelSet *k);
bool kernels_bf16(int feat, int plm, int wide, KernelSet *k);

void launch_relabel(const DevDomain *doms, const PItem *items, int nitems, hipStream_t s);
void launch_near_tiles(const DevDomain *dom, int ntiles, int kstep, hipStream_t s);
void launch_masks_full(const DevDomain *dom, int nx, int ny, hipStream_t s);
void launch_mass_final(const DevDomain *doms, int ndom, const double *alt, double *alt_out,
                       hipStream_t s);
void launch_normals(uint32_t k0, uint32_t k1, uint32_t step, uint32_t node0, uint32_t count,
                    bool hw, float *out, hipStream_t s);
void launch_advance(const DevDomain *doms, int ndom, int n, hipStream_t s);

}  // namespace lbk
