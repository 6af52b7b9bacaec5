// Storage-independent kernels: initial particle labels, mass total,
// noise diagnostic, step counter.
#define LBK_COMMON_KERNELS 1
#include "aux_impl.h"
#include "launch.h"
#include "particles_impl.h"

namespace lbk {

void launch_relabel(const DevDomain *doms, const PItem *items, int nitems, hipStream_t s) {
  hipLaunchKernelGGL(k_relabel, dim3(nitems), dim3(256), 0, s, doms, items);
}
void launch_near_tiles(const DevDomain *dom, int ntiles, int kstep, hipStream_t s) {
  hipLaunchKernelGGL(k_near_tiles, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, dom,
                     kstep);
}
void launch_masks_full(const DevDomain *dom, int nx, int ny, hipStream_t s) {
  const long long n = (long long)nx * ny;
  hipLaunchKernelGGL(k_masks_full, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dom);
}
void launch_mass_final(const DevDomain *doms, int ndom, const double *alt, double *alt_out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_mass_final, dim3(ndom), dim3(64), 0, s, doms, alt, alt_out);
}
void launch_normals(uint32_t k0, uint32_t k1, uint32_t step, uint32_t node0, uint32_t count,
                    bool hw, float *out, hipStream_t s) {
  if (hw)
    hipLaunchKernelGGL(k_normals<true>, dim3((count + 255) / 256), dim3(256), 0, s, k0, k1, step,
                       node0, count, out);
  else
    hipLaunchKernelGGL(k_normals<false>, dim3((count + 255) / 256), dim3(256), 0, s, k0, k1, step,
                       node0, count, out);
}
void launch_advance(const DevDomain *doms, int ndom, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3((ndom + 63) / 64), dim3(64), 0, s, doms, ndom, n);
}

}  // namespace lbk
