// lb3_api.hip -- C ABI of the D3Q19 / D3Q27 domains (declared in include/lb.h):
// validation, workspace layout, launch sequence, host transfers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lb.h"
#include "sweep3_impl.h"

using namespace lbk3;

namespace lbk {
// records msg as lb_last_error() and returns s (lb_api.hip)
lb_status lb_fail(lb_status s, const std::string &msg);
// the same without throwing (lb_api.hip)
lb_status lb_fail_nothrow(lb_status s, const char *msg) noexcept;
}

namespace {

lb_status fail3(lb_status s, const std::string &msg) { return lbk::lb_fail(s, msg); }

#define HIPCHK3(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail3(LB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

// nodes per host-transfer band (initial fields, moments, populations)
constexpr long long BAND = 262144;

struct Header3 {
  uint64_t tstep;
  uint32_t health, pad;
  double mass;
};

struct Layout3 {
  int pitch = 0;
  size_t desc = 0, hdr = 0, f0 = 0, f1 = 0, nodew = 0, mask = 0, partials = 0, stage = 0, total = 0;
  bool solids = false;
};

int q_of(const lb3_domain_desc *d) { return d->lattice == LB3_D3Q27 ? 27 : 19; }
size_t elem_of(int storage) { return storage == LB_F64 ? 8 : storage == LB_F32 ? 4 : 2; }

Layout3 layout3(const lb3_domain_desc *d) {
  Layout3 L;
  L.pitch = (d->nx + 63) / 64 * 64;
  const size_t nodes = (size_t)d->nz * d->ny * L.pitch;
  const size_t fbytes = (size_t)q_of(d) * nodes * elem_of(d->storage);
  L.solids = d->obstacles || d->wall_x || d->wall_y || d->wall_z;
  size_t o = 0;
  L.desc = o; o += al256(sizeof(Dom3));
  L.hdr = o; o += al256(sizeof(Header3));
  L.f0 = o; o += al256(fbytes);
  L.f1 = o; o += al256(fbytes);
  L.nodew = o; if (L.solids) o += al256(nodes * 4);
  L.mask = o; if (L.solids) o += al256(nodes);
  L.partials = o; o += al256((size_t)d->nz * 8);
  L.stage = o; o += al256((size_t)q_of(d) * BAND * 8);
  L.total = o;
  return L;
}

lb_status validate3(const lb3_domain_desc *d) {
  if (!d) return fail3(LB_EINVAL, "desc is null");
  if (d->abi_version != LB_ABI_VERSION) return fail3(LB_EINVAL, "abi_version mismatch");
  if (d->nx < 3 || d->ny < 3 || d->nz < 3 || d->nx > 4096 || d->ny > 4096 || d->nz > 4096)
    return fail3(LB_EINVAL, "nx, ny, nz must be in [3, 4096]");
  if (d->storage != LB_F64 && d->storage != LB_F32 && d->storage != LB_F16_DELTA &&
      d->storage != LB_BF16_DELTA)
    return fail3(LB_EINVAL, "storage must be LB_F64, LB_F32, LB_F16_DELTA or LB_BF16_DELTA");
  if (d->lattice != LB3_D3Q19 && d->lattice != LB3_D3Q27)
    return fail3(LB_EINVAL, "lattice must be LB3_D3Q19 or LB3_D3Q27");
  if (d->rounding != LB_ROUND_NEAREST && d->rounding != LB_ROUND_STOCHASTIC)
    return fail3(LB_EINVAL, "rounding must be LB_ROUND_NEAREST or LB_ROUND_STOCHASTIC");
  if (d->rounding == LB_ROUND_STOCHASTIC && d->storage != LB_F16_DELTA &&
      d->storage != LB_BF16_DELTA)
    return fail3(LB_EINVAL, "stochastic rounding needs LB_F16_DELTA or LB_BF16_DELTA storage");
  if (!d->power_law && !(d->tau > 0.5)) return fail3(LB_EINVAL, "tau must be > 1/2");
  if (d->power_law && (!(d->tau_min > 0.5) || !(d->tau_max >= d->tau_min) || !(d->n_index > 0.0) ||
                       !(d->K > 0.0) || !std::isfinite(d->n_index) || !std::isfinite(d->K) ||
                       !std::isfinite(d->tau_max)))
    return fail3(LB_EINVAL, "power law needs n > 0, K > 0, 1/2 < tau_min <= tau_max");
  if (d->collision != LB3_BGK && d->collision != LB3_TRT)
    return fail3(LB_EINVAL, "collision must be LB3_BGK or LB3_TRT");
  if (d->collision == LB3_TRT && !(d->magic > 0.0 && std::isfinite(d->magic)))
    return fail3(LB_EINVAL, "TRT magic number must be finite and > 0");
  if (!(d->kT >= 0.0) || !std::isfinite(d->kT)) return fail3(LB_EINVAL, "kT must be finite and >= 0");
  if (d->kT > 0.0 && (double)d->nx * d->ny * d->nz >= 4294967296.0)
    return fail3(LB_EUNSUPPORTED, "thermal noise needs fewer than 2^32 nodes");
  if (!(d->rho0 > 0.0) || !std::isfinite(d->rho0)) return fail3(LB_EINVAL, "rho0 must be > 0");
  if (!std::isfinite(d->gx) || !std::isfinite(d->gy) || !std::isfinite(d->gz))
    return fail3(LB_EINVAL, "g not finite");
  if (d->init_kind != LB_INIT_REST && d->init_kind != LB_INIT_FIELDS)
    return fail3(LB_EINVAL, "bad init_kind");
  if (d->init_kind == LB_INIT_FIELDS && (!d->init_rho || !d->init_ux || !d->init_uy || !d->init_uz))
    return fail3(LB_EINVAL, "LB_INIT_FIELDS needs init_rho, init_ux, init_uy, init_uz");
  return LB_OK;
}

unsigned blocks_of(long long n) { return (unsigned)((n + 255) / 256); }

// launches kernel template K<storage, q> for storage format st and lattice
// size q (both validated)
#define LB3_DISPATCH_Q(st, Qv, K, ...)                                            \
  do {                                                                            \
    switch (st) {                                                                 \
      case LB_F64: hipLaunchKernelGGL((K<0, Qv>), __VA_ARGS__); break;            \
      case LB_F32: hipLaunchKernelGGL((K<1, Qv>), __VA_ARGS__); break;            \
      case LB_F16_DELTA: hipLaunchKernelGGL((K<2, Qv>), __VA_ARGS__); break;      \
      default: hipLaunchKernelGGL((K<3, Qv>), __VA_ARGS__); break;                \
    }                                                                             \
  } while (0)
#define LB3_DISPATCH(d, K, ...)                                                   \
  do {                                                                            \
    if ((d)->q == 27) LB3_DISPATCH_Q((d)->desc.storage, 27, K, __VA_ARGS__);      \
    else LB3_DISPATCH_Q((d)->desc.storage, 19, K, __VA_ARGS__);                   \
  } while (0)

}  // namespace

struct lb3_domain {
  lb3_domain_desc desc{};
  Layout3 L;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  Dom3 hd{};
  int64_t t = 0;
  bool wide = false;               // the sweep takes 64-bit byte offsets
  int q = 19;                      // lattice velocities
  std::vector<uint8_t> host_mask;  // [nz][ny][pitch]: walls and obstacles
  Dom3 *ddesc() const { return (Dom3 *)(ws + L.desc); }
  Header3 *dhdr() const { return (Header3 *)(ws + L.hdr); }
  long long nodes() const { return (long long)desc.nx * desc.ny * desc.nz; }
};

namespace {

lb_status check_health3(lb3_domain *d) {
  uint32_t h = 0;
  HIPCHK3(hipMemcpyAsync(&h, &d->dhdr()->health, sizeof(h), hipMemcpyDeviceToHost, d->stream));
  HIPCHK3(hipStreamSynchronize(d->stream));
  if (h) return fail3(LB_EUNSTABLE, "device latched: non-finite density");
  return LB_OK;
}

// mask of walls and obstacles to the device, and the node words from it
lb_status upload_solids(lb3_domain *d) {
  HIPCHK3(hipMemcpyAsync(d->ws + d->L.mask, d->host_mask.data(), d->host_mask.size(),
                         hipMemcpyHostToDevice, d->stream));
  const uint8_t *dm = (const uint8_t *)(d->ws + d->L.mask);
  if (d->q == 27)
    hipLaunchKernelGGL(k_words3<27>, dim3(blocks_of(d->nodes())), dim3(256), 0, d->stream, d->ddesc(),
                       dm);
  else
    hipLaunchKernelGGL(k_words3<19>, dim3(blocks_of(d->nodes())), dim3(256), 0, d->stream, d->ddesc(),
                       dm);
  HIPCHK3(hipGetLastError());
  HIPCHK3(hipStreamSynchronize(d->stream));
  return LB_OK;
}

// initial state from host fields (null: rest), band by band through the
// staging area
lb_status init3(lb3_domain *d, const double *rho, const double *ux, const double *uy,
                const double *uz) {
  const long long n = d->nodes();
  double *st = (double *)(d->ws + d->L.stage);
  for (long long n0 = 0; n0 < n; n0 += BAND) {
    const long long cnt = std::min(BAND, n - n0);
    const double *a[4] = {nullptr, nullptr, nullptr, nullptr};
    if (rho) {
      const double *h[4] = {rho, ux, uy, uz};
      for (int k = 0; k < 4; ++k) {
        HIPCHK3(hipMemcpyAsync(st + k * BAND, h[k] + n0, cnt * 8, hipMemcpyHostToDevice, d->stream));
        a[k] = st + k * BAND;
      }
    }
    LB3_DISPATCH(d, k_init3, dim3(blocks_of(cnt)), dim3(256), 0, d->stream,
                 d->ddesc(), a[0], a[1], a[2], a[3], n0, cnt);
    HIPCHK3(hipGetLastError());
    HIPCHK3(hipStreamSynchronize(d->stream));
  }
  return LB_OK;
}

lb_status push_desc3(lb3_domain *d) {
  HIPCHK3(hipMemcpyAsync(d->ddesc(), &d->hd, sizeof(Dom3), hipMemcpyHostToDevice, d->stream));
  HIPCHK3(hipStreamSynchronize(d->stream));
  return LB_OK;
}

}  // namespace

// Every entry point runs its body through LB_GUARDED, so that no C++
// exception (a failed host allocation, say) crosses the C ABI.
#define LB_GUARDED(call)                                                           \
  try {                                                                            \
    return call;                                                                   \
  } catch (const std::bad_alloc &) {                                               \
    return lbk::lb_fail_nothrow(LB_ENOMEM, "host memory allocation failed");       \
  } catch (...) {                                                                  \
    return lbk::lb_fail_nothrow(LB_EHIP, "unexpected internal error");             \
  }

namespace {

template <int ST, int Q, bool PL, int NZ>
void launch_sweep3_qn(const lb3_domain *d, unsigned blocks, int k) {
  const dim3 g(blocks), b(256);
  if (d->L.solids) {
    if (d->wide)
      hipLaunchKernelGGL((k_sweep3<ST, true, true, Q, PL, NZ>), g, b, 0, d->stream, d->ddesc(), k);
    else
      hipLaunchKernelGGL((k_sweep3<ST, true, false, Q, PL, NZ>), g, b, 0, d->stream, d->ddesc(), k);
  } else {
    if (d->wide)
      hipLaunchKernelGGL((k_sweep3<ST, false, true, Q, PL, NZ>), g, b, 0, d->stream, d->ddesc(), k);
    else
      hipLaunchKernelGGL((k_sweep3<ST, false, false, Q, PL, NZ>), g, b, 0, d->stream, d->ddesc(), k);
  }
}
template <int ST, int Q, bool PL> void launch_sweep3_q(const lb3_domain *d, unsigned blocks, int k) {
  // noise kind: none, with BGK, with TRT (the last needs more registers)
  if (!d->hd.noise) launch_sweep3_qn<ST, Q, PL, 0>(d, blocks, k);
  else if (d->hd.trt) launch_sweep3_qn<ST, Q, PL, 2>(d, blocks, k);
  else launch_sweep3_qn<ST, Q, PL, 1>(d, blocks, k);
}
template <int ST> void launch_sweep3_st(const lb3_domain *d, unsigned blocks, int k) {
  const bool pl = d->desc.power_law != 0;
  if (d->q == 27) {
    if (pl) launch_sweep3_q<ST, 27, true>(d, blocks, k);
    else launch_sweep3_q<ST, 27, false>(d, blocks, k);
  } else {
    if (pl) launch_sweep3_q<ST, 19, true>(d, blocks, k);
    else launch_sweep3_q<ST, 19, false>(d, blocks, k);
  }
}

void launch_sweep3(const lb3_domain *d, unsigned blocks, int k) {
  switch (d->desc.storage) {
    case LB_F64: launch_sweep3_st<0>(d, blocks, k); break;
    case LB_F32: launch_sweep3_st<1>(d, blocks, k); break;
    case LB_F16_DELTA: launch_sweep3_st<2>(d, blocks, k); break;
    default: launch_sweep3_st<3>(d, blocks, k); break;
  }
}

}  // namespace

extern "C" {

static lb_status lb3_workspace_bytes_impl(const lb3_domain_desc *desc, size_t *bytes) {
  if (!bytes) return fail3(LB_EINVAL, "bytes is null");
  lb_status s = validate3(desc);
  if (s != LB_OK) return s;
  *bytes = layout3(desc).total;
  return LB_OK;
}

lb_status lb3_workspace_bytes(const lb3_domain_desc *desc, size_t *bytes) {
  LB_GUARDED(lb3_workspace_bytes_impl(desc, bytes));
}

static lb_status lb3_create_domain_impl(const lb3_domain_desc *desc, void *dev_workspace, size_t bytes,
                                        void *hip_stream, lb3_domain **out) {
  if (!out) return fail3(LB_EINVAL, "out is null");
  *out = nullptr;
  lb_status s = validate3(desc);
  if (s != LB_OK) return s;
  if (!dev_workspace || ((uintptr_t)dev_workspace & 255))
    return fail3(LB_EINVAL, "workspace must be non-null and 256-byte aligned");
  const Layout3 L = layout3(desc);
  if (bytes < L.total) return fail3(LB_ENOMEM, "workspace smaller than lb3_workspace_bytes");
  lb3_domain *d = new lb3_domain();
  d->desc = *desc;
  d->desc.init_rho = d->desc.init_ux = d->desc.init_uy = d->desc.init_uz = nullptr;
  d->L = L;
  d->ws = (char *)dev_workspace;
  d->stream = (hipStream_t)hip_stream;
  Dom3 &h = d->hd;
  h.f[0] = d->ws + L.f0;
  h.f[1] = d->ws + L.f1;
  h.nodew = L.solids ? (uint32_t *)(d->ws + L.nodew) : nullptr;
  h.tstep = &d->dhdr()->tstep;
  h.health = &d->dhdr()->health;
  h.partials = (double *)(d->ws + L.partials);
  h.mass = &d->dhdr()->mass;
  h.nx = desc->nx;
  h.ny = desc->ny;
  h.nz = desc->nz;
  h.pitch = L.pitch;
  h.storage = desc->storage;
  // 32-bit byte offsets while the q population planes stay below 2^32 bytes
  d->q = q_of(desc);
  d->wide = (double)d->q * d->desc.nz * d->desc.ny * L.pitch *
                (desc->storage == LB_F64 ? 8 : desc->storage == LB_F32 ? 4 : 2) >=
            4294967296.0;
  h.sr = desc->rounding == LB_ROUND_STOCHASTIC ? 1 : 0;
  h.key0 = (uint32_t)desc->seed;
  h.key1 = (uint32_t)(desc->seed >> 32);
  h.tiles_x = (desc->nx + 63) / 64;
  h.tiles_y = (desc->ny + 3) / 4;
  h.rho0 = desc->rho0;
  // with the power law tau is the local tau*; the domain-wide values below
  // are those of tau_min (unused by the sweep)
  h.tau = desc->power_law ? desc->tau_min : desc->tau;
  h.pl = desc->power_law ? 1 : 0;
  h.pl_n = desc->n_index;
  h.pl_K = desc->K;
  h.tau_min = desc->tau_min;
  h.tau_max = desc->tau_max;
  h.magic = desc->magic;
  h.pl_n_f = (float)h.pl_n;
  h.pl_K_f = (float)h.pl_K;
  h.tau_min_f = (float)h.tau_min;
  h.tau_max_f = (float)h.tau_max;
  h.magic_f = (float)h.magic;
  h.omega = 1.0 / h.tau;
  h.trt = desc->collision == LB3_TRT ? 1 : 0;
  h.noise = desc->kT > 0.0 ? 1 : 0;
  h.kT = desc->kT;
  h.kT_f = (float)desc->kT;
  h.tau_m = h.trt ? 0.5 + desc->magic / (h.tau - 0.5) : h.tau;
  h.omega_m = 1.0 / h.tau_m;
  h.tau_m_f = (float)h.tau_m;
  h.omega_m_f = (float)h.omega_m;
  {
    // 16-bit storage: coefficients in the stored scaling (K w of every
    // moving direction: 8/9 on D3Q19, 32/27 on D3Q27)
    const double f = h.trt ? 1.0 : h.omega;
    const double kw = d->q == 27 ? 32.0 / 27.0 : 8.0 / 9.0;
    h.s_cw = (float)(f * kw);
    h.s_cq = (float)(4.5 * f * kw);
    h.s_cl = (float)(3.0 * f * kw);
    h.s_om0 = (float)f;
    h.keep_f = (float)(1.0 - h.omega);
  }
  h.gx = desc->gx;
  h.gy = desc->gy;
  h.gz = desc->gz;
  h.rho0_f = (float)h.rho0;
  h.tau_f = (float)h.tau;
  h.omega_f = (float)h.omega;
  h.gx_f = (float)h.gx;
  h.gy_f = (float)h.gy;
  h.gz_f = (float)h.gz;
  auto bail = [&](lb_status st) {
    delete d;
    return st;
  };
  Header3 zero{};
  if (hipMemcpyAsync(d->dhdr(), &zero, sizeof(zero), hipMemcpyHostToDevice, d->stream) != hipSuccess)
    return bail(fail3(LB_EHIP, "header upload failed"));
  if ((s = push_desc3(d)) != LB_OK) return bail(s);
  if (L.solids) {
    d->host_mask.assign((size_t)desc->nz * desc->ny * L.pitch, 0);
    for (int z = 0; z < desc->nz; ++z)
      for (int y = 0; y < desc->ny; ++y)
        for (int x = 0; x < desc->nx; ++x) {
          const bool wall = (desc->wall_x && (x == 0 || x == desc->nx - 1)) ||
                            (desc->wall_y && (y == 0 || y == desc->ny - 1)) ||
                            (desc->wall_z && (z == 0 || z == desc->nz - 1));
          d->host_mask[((size_t)z * desc->ny + y) * L.pitch + x] = wall ? 1 : 0;
        }
    if ((s = upload_solids(d)) != LB_OK) return bail(s);
  }
  if ((s = init3(d, desc->init_kind == LB_INIT_FIELDS ? desc->init_rho : nullptr, desc->init_ux,
                 desc->init_uy, desc->init_uz)) != LB_OK)
    return bail(s);
  *out = d;
  return LB_OK;
}

lb_status lb3_create_domain(const lb3_domain_desc *desc, void *dev_workspace, size_t bytes,
                            void *hip_stream, lb3_domain **out) {
  LB_GUARDED(lb3_create_domain_impl(desc, dev_workspace, bytes, hip_stream, out));
}

static lb_status lb3_set_obstacles_impl(lb3_domain *d, const uint8_t *mask, size_t n) {
  if (!d || !mask) return fail3(LB_EINVAL, "null argument");
  if (!d->desc.obstacles) return fail3(LB_ESTATE, "domain was created without obstacles");
  if (n != (size_t)d->nodes()) return fail3(LB_EINVAL, "mask size must be nx*ny*nz");
  const lb3_domain_desc &c = d->desc;
  const int pitch = d->L.pitch;
  for (int z = 0; z < c.nz; ++z)
    for (int y = 0; y < c.ny; ++y)
      for (int x = 0; x < c.nx; ++x) {
        const bool wall = (c.wall_x && (x == 0 || x == c.nx - 1)) ||
                          (c.wall_y && (y == 0 || y == c.ny - 1)) ||
                          (c.wall_z && (z == 0 || z == c.nz - 1));
        d->host_mask[((size_t)z * c.ny + y) * pitch + x] =
            (wall || mask[((size_t)z * c.ny + y) * c.nx + x]) ? 1 : 0;
      }
  lb_status s = upload_solids(d);
  if (s != LB_OK) return s;
  // solid nodes hold zero deviations in the current state
  return LB_OK;
}

lb_status lb3_set_obstacles(lb3_domain *d, const uint8_t *mask, size_t n) {
  LB_GUARDED(lb3_set_obstacles_impl(d, mask, n));
}

static lb_status lb3_step_impl(lb3_domain *d, int64_t nsteps) {
  if (!d) return fail3(LB_EINVAL, "null domain");
  if (nsteps < 0) return fail3(LB_EINVAL, "nsteps < 0");
  const unsigned blocks = (unsigned)(d->hd.tiles_x * d->hd.tiles_y * d->desc.nz);
  for (int64_t k0 = 0; k0 < nsteps; k0 += 1024) {
    const int c = (int)std::min<int64_t>(1024, nsteps - k0);
    for (int k = 0; k < c; ++k) {
      launch_sweep3(d, blocks, k);
    }
    hipLaunchKernelGGL(k_advance3, dim3(1), dim3(1), 0, d->stream, d->ddesc(), c);
    HIPCHK3(hipGetLastError());
  }
  d->t += nsteps;
  return LB_OK;
}

lb_status lb3_step(lb3_domain *d, int64_t nsteps) {
  LB_GUARDED(lb3_step_impl(d, nsteps));
}

static lb_status lb3_moments_impl(lb3_domain *d, double *rho, double *ux, double *uy, double *uz) {
  if (!d || !rho || !ux || !uy || !uz) return fail3(LB_EINVAL, "null argument");
  const long long n = d->nodes();
  double *st = (double *)(d->ws + d->L.stage);
  double *h[4] = {rho, ux, uy, uz};
  for (long long n0 = 0; n0 < n; n0 += BAND) {
    const long long cnt = std::min(BAND, n - n0);
    LB3_DISPATCH(d, k_moments3, dim3(blocks_of(cnt)), dim3(256), 0, d->stream,
                 d->ddesc(), st, n0, cnt);
    HIPCHK3(hipGetLastError());
    for (int k = 0; k < 4; ++k)
      HIPCHK3(hipMemcpyAsync(h[k] + n0, st + k * cnt, cnt * 8, hipMemcpyDeviceToHost, d->stream));
    HIPCHK3(hipStreamSynchronize(d->stream));
  }
  return check_health3(d);
}

lb_status lb3_moments(lb3_domain *d, double *rho, double *ux, double *uy, double *uz) {
  LB_GUARDED(lb3_moments_impl(d, rho, ux, uy, uz));
}

static lb_status lb3_get_populations_impl(lb3_domain *d, double *f) {
  if (!d || !f) return fail3(LB_EINVAL, "null argument");
  const long long n = d->nodes();
  double *st = (double *)(d->ws + d->L.stage);
  for (long long n0 = 0; n0 < n; n0 += BAND) {
    const long long cnt = std::min(BAND, n - n0);
    LB3_DISPATCH(d, k_export3, dim3(blocks_of(cnt)), dim3(256), 0, d->stream,
                 d->ddesc(), st, n0, cnt);
    HIPCHK3(hipGetLastError());
    for (int i = 0; i < d->q; ++i)
      HIPCHK3(hipMemcpyAsync(f + (size_t)i * n + n0, st + (size_t)i * cnt, cnt * 8,
                             hipMemcpyDeviceToHost, d->stream));
    HIPCHK3(hipStreamSynchronize(d->stream));
  }
  return check_health3(d);
}

lb_status lb3_get_populations(lb3_domain *d, double *f) {
  LB_GUARDED(lb3_get_populations_impl(d, f));
}

static lb_status lb3_mass_impl(lb3_domain *d, double *total) {
  if (!d || !total) return fail3(LB_EINVAL, "null argument");
  LB3_DISPATCH(d, k_mass3_partial, dim3(d->desc.nz), dim3(256), 0, d->stream,
               d->ddesc());
  hipLaunchKernelGGL(k_mass3_final, dim3(1), dim3(64), 0, d->stream, d->ddesc());
  HIPCHK3(hipGetLastError());
  HIPCHK3(hipMemcpyAsync(total, &d->dhdr()->mass, 8, hipMemcpyDeviceToHost, d->stream));
  HIPCHK3(hipStreamSynchronize(d->stream));
  return check_health3(d);
}

lb_status lb3_mass(lb3_domain *d, double *total) {
  LB_GUARDED(lb3_mass_impl(d, total));
}

static lb_status lb3_time_impl(lb3_domain *d, int64_t *t) {
  if (!d || !t) return fail3(LB_EINVAL, "null argument");
  *t = d->t;
  return LB_OK;
}

lb_status lb3_time(lb3_domain *d, int64_t *t) {
  LB_GUARDED(lb3_time_impl(d, t));
}

static lb_status lb3_set_option_impl(lb3_domain *d, int32_t option, int64_t value) {
  if (!d) return fail3(LB_EINVAL, "null domain");
  switch (option) {
    case LB3_OPT_WIDE_OFFSETS: {
      if (value != 0 && value != 1) return fail3(LB_EINVAL, "LB3_OPT_WIDE_OFFSETS takes 0 or 1");
      const Layout3 &L = d->L;
      const size_t e = d->desc.storage == LB_F64 ? 8 : d->desc.storage == LB_F32 ? 4 : 2;
      const bool need = (double)d->q * d->desc.nz * d->desc.ny * L.pitch * e >= 4294967296.0;
      if (!value && need)
        return fail3(LB_EINVAL, "population buffer reaches 2^32 bytes: offsets must stay 64-bit");
      d->wide = value != 0;
      return LB_OK;
    }
  }
  return fail3(LB_EINVAL, "unknown option of a 3D domain");
}

lb_status lb3_set_option(lb3_domain *d, int32_t option, int64_t value) {
  LB_GUARDED(lb3_set_option_impl(d, option, value));
}

static lb_status lb3_destroy_domain_impl(lb3_domain *d) {
  if (!d) return fail3(LB_EINVAL, "null domain");
  (void)hipStreamSynchronize(d->stream);
  delete d;
  return LB_OK;
}

lb_status lb3_destroy_domain(lb3_domain *d) {
  LB_GUARDED(lb3_destroy_domain_impl(d));
}

}  // extern "C"
