// aux_impl.h -- reductions and data movement around the sweep: FP64 mass
// check with a non-finite latch, moments, population export/import, the
// noise-normal diagnostic and the step counter.
#pragma once

#include "lb_device.h"

namespace lbk {

__device__ __forceinline__ bool node_is_solid(const DevDomain &D, int x, int y) {
  if (D.label) return D.label[(size_t)y * D.pitch + x] == LBL_SOLID;
  return (D.bc_y == BC_WALL && (y == 0 || y == D.ny - 1)) ||
         (D.bc_x == BC_WALL && (x == 0 || x == D.nx - 1));
}

// Partial FP64 sums of rho over the non-solid nodes of every domain of a
// launch: domain d owns blocks prefix[d] .. prefix[d+1]-1 (its mass_blocks);
// local block k sums rows k, k + mass_blocks, ..., each row with the 256
// threads striding along x, in a fixed order into the domain's partials[k]
// (or into alt[k] when alt is given: one domain, ndom == 1).
template <int ST>
__global__ __launch_bounds__(256) void k_mass_partial(const DevDomain *__restrict__ doms,
                                                      const int *__restrict__ prefix, int ndom,
                                                      double *alt) {
  using S = Store<ST>;
  using T = typename S::T;
  __shared__ double red[4];
  const int b = (int)blockIdx.x;
  const int dix = ndom == 1 ? 0 : find_domain(prefix, ndom, b);
  const DevDomain &D = doms[dix];
  const int local = b - prefix[dix];
  const uint64_t T0 = *D.tstep;
  const T *src = (const T *)D.f[T0 & 1];
  const size_t plane = (size_t)D.ny * D.pitch;
  double acc = 0.0;
  for (int y = local; y < D.ny; y += D.mass_blocks) {
    for (int x = (int)threadIdx.x; x < D.nx; x += 256) {
      if (node_is_solid(D, x, y)) continue;
      const size_t here = (size_t)y * D.pitch + x;
      double r = 0.0;
#pragma unroll
      for (int i = 0; i < 9; ++i) r += (double)S::load(src + i * plane, here, i);
      acc += D.rho0 + r;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) (alt ? alt : D.partials)[local] = (red[0] + red[1]) + (red[2] + red[3]);
}

#ifdef LBK_COMMON_KERNELS
// Total of each domain's partials, one wave per domain in a fixed order (lane
// l sums partials l, l + 64, ...; then a butterfly over the lanes).  Latches a
// non-finite total, and a total that drifts from the reference by more than
// the relative tolerance when one is set.  With alt (one domain) the
// partials are read from alt and the total is also written to *alt_out.
__global__ __launch_bounds__(64) void k_mass_final(const DevDomain *__restrict__ doms,
                                                   const double *alt, double *alt_out) {
  const DevDomain &D = doms[blockIdx.x];
  const double *part = alt ? alt : D.partials;
  double s = 0.0;
  for (int i = (int)threadIdx.x; i < D.mass_blocks; i += 64) s += part[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) {
    *D.mass_out = s;
    if (alt_out) *alt_out = s;
    if (!(fabs(s) < 1e300)) atomicOr(D.health, HEALTH_NONFINITE);
    const double ref = D.mass_ctl[0], tol = D.mass_ctl[1];
    if (tol > 0.0 && !(fabs(s - ref) <= tol * fabs(ref))) atomicOr(D.health, HEALTH_MASS_DRIFT);
  }
}
#endif  // LBK_COMMON_KERNELS

// rho and u = j/rho + g/2 of the pre-collision state f(T), recovered from
// f*(T): collision keeps rho and adds rho g to j.  Band rows [row0, row0+nrows).
template <int ST>
__global__ __launch_bounds__(256) void k_moments(const DevDomain *__restrict__ Dp, double *rho_o,
                                                 double *ux_o, double *uy_o, int row0, int nrows) {
  using S = Store<ST>;
  using T = typename S::T;
  const DevDomain &D = *Dp;
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n >= (long long)nrows * D.nx) return;
  const int yl = (int)(n / D.nx), x = (int)(n - (long long)yl * D.nx);
  const int y = row0 + yl;
  if (node_is_solid(D, x, y)) {
    rho_o[n] = 0.0; ux_o[n] = 0.0; uy_o[n] = 0.0;
    return;
  }
  const uint64_t T0 = *D.tstep;
  const T *src = (const T *)D.f[T0 & 1];
  const size_t plane = (size_t)D.ny * D.pitch;
  const uint32_t here = (uint32_t)y * D.pitch + x;
  double dr = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double v = (double)S::load(src + i * plane, here, i);
    dr += v;
    jx += v * cx(i);
    jy += v * cy(i);
  }
  const double rho = D.rho0 + dr;
  rho_o[n] = rho;
  ux_o[n] = jx / rho - 0.5 * D.gx;
  uy_o[n] = jy / rho - 0.5 * D.gy;
}

// Mirror slots of the index walls of a label-free domain in the current
// buffer: for every fluid node x whose pull along i comes from a wall node
// s = x - e_i, slot i of s holds x's own opposite population (what that pull
// bounces back), copied bit for bit.
template <int ST>
__global__ __launch_bounds__(256) void k_mirror(const DevDomain *__restrict__ Dp) {
  using T = typename Store<ST>::T;
  const DevDomain &D = *Dp;
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n >= (long long)D.ny * D.nx) return;
  const int y = (int)(n / D.nx), x = (int)(n - (long long)y * D.nx);
  const size_t here = (size_t)y * D.pitch + x;
  const bool perx = D.bc_x == BC_PERIODIC, pery = D.bc_y == BC_PERIODIC;
  if (node_is_solid(D, x, y)) return;
  T *f = (T *)D.f[*D.tstep & 1];
  const size_t plane = (size_t)D.ny * D.pitch;
  for (int i = 1; i < 9; ++i) {
    int sx, sy;
    if (!source_of(D.nx, D.ny, perx, pery, x, y, i, sx, sy) || !node_is_solid(D, sx, sy)) continue;
    f[i * plane + (size_t)sy * D.pitch + sx] = f[opp(i) * plane + here];
  }
}

// Export / import of the stored deviations as FP64, band layout [9][nrows][nx].
template <int ST>
__global__ __launch_bounds__(256) void k_export(const DevDomain *__restrict__ Dp, double *out,
                                                int row0, int nrows) {
  using S = Store<ST>;
  using T = typename S::T;
  const DevDomain &D = *Dp;
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n >= (long long)nrows * D.nx) return;
  const int yl = (int)(n / D.nx), x = (int)(n - (long long)yl * D.nx);
  const uint64_t T0 = *D.tstep;
  const T *src = (const T *)D.f[T0 & 1];
  const size_t plane = (size_t)D.ny * D.pitch;
  const uint32_t here = (uint32_t)(row0 + yl) * D.pitch + x;
  const bool solid = node_is_solid(D, x, row0 + yl);  // never written by the sweep
  for (int i = 0; i < 9; ++i)
    out[(size_t)i * nrows * D.nx + n] = solid ? 0.0 : (double)S::load(src + i * plane, here, i);
}

template <int ST>
__global__ __launch_bounds__(256) void k_import(const DevDomain *__restrict__ Dp, const double *in,
                                                int row0, int nrows) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  const DevDomain &D = *Dp;
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n >= (long long)nrows * D.nx) return;
  const int yl = (int)(n / D.nx), x = (int)(n - (long long)yl * D.nx);
  const uint64_t T0 = *D.tstep;
  T *dst = (T *)D.f[T0 & 1];
  const size_t plane = (size_t)D.ny * D.pitch;
  const uint32_t here = (uint32_t)(row0 + yl) * D.pitch + x;
  for (int i = 0; i < 9; ++i)
    S::put(dst + i * plane, here, i, (R)in[(size_t)i * nrows * D.nx + n], 0u);
}

#ifdef LBK_COMMON_KERNELS
// Static node words of every node (after the label plane is written).
__global__ __launch_bounds__(256) void k_masks_full(const DevDomain *__restrict__ Dp) {
  const DevDomain &D = *Dp;
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n >= (long long)D.ny * D.nx) return;
  const int y = (int)(n / D.nx), x = (int)(n - (long long)y * D.nx);
  const bool perx = D.bc_x == BC_PERIODIC, pery = D.bc_y == BC_PERIODIC;
  const size_t here = (size_t)y * D.pitch + x;
  D.nodew[here] = node_word(D.label, D.nx, D.ny, D.pitch, perx, pery, x, y);
}

template <bool HW>
__global__ __launch_bounds__(256) void k_normals(uint32_t k0, uint32_t k1, uint32_t step,
                                                 uint32_t node0, uint32_t count, float *out) {
  const uint32_t n = blockIdx.x * 256 + threadIdx.x;
  if (n >= count) return;
  float th[6];
  noise_normals<HW>(k0, k1, node0 + n, step, th);
#pragma unroll
  for (int k = 0; k < 6; ++k) out[(size_t)n * 6 + k] = th[k];
}

// Advance the step counters of a batch's domains after n captured steps.
__global__ void k_advance(const DevDomain *__restrict__ doms, int ndom, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ndom) *doms[i].tstep += (uint64_t)n;
}
#endif  // LBK_COMMON_KERNELS

}  // namespace lbk
