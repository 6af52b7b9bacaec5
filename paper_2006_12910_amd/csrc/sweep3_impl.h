// sweep3_impl.h -- the D3Q19 variant of the fused stream-collide sweep (the
// three-dimensional lattice the paper names as its next step, Sec. 8): BGK
// collision with the velocity-shift body force of Sec. 2, pull streaming
// with periodic wrap and halfway bounce-back on solid nodes, FP64 or FP32
// storage of the deviations d_i = f_i - w_i rho0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbk3 {

// D3Q19: rest, six axis velocities, twelve edge velocities; opposite
// velocities at (i, i + 1) for odd i.  Weights 1/3, 1/18, 1/36.
__host__ __device__ constexpr int ex(int i) {
  return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
       : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int ey(int i) {
  return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
       : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int ez(int i) {
  return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
       : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
static_assert(ex(1) == 1 && ex(2) == -1 && ey(3) == 1 && ey(4) == -1 && ez(5) == 1 && ez(6) == -1,
              "axis velocities");
static_assert(ex(7) == 1 && ey(7) == 1 && ex(8) == -1 && ey(8) == -1, "edge pair 7/8");
static_assert(ex(17) == 0 && ey(17) == 1 && ez(17) == -1 && ey(18) == -1 && ez(18) == 1,
              "edge pair 17/18");

constexpr uint32_t NODE_SOLID3 = 0x80000000u;  // node word: the node is solid

struct Dom3 {
  void *f[2];          // populations [19][nz][ny][pitch], deviations
  uint32_t *nodew;     // [nz][ny][pitch]: NODE_SOLID3, or bit i-1 when the
                       // source x - e_i is solid; null without solids
  uint64_t *tstep;
  uint32_t *health;
  double *partials;    // FP64 density partial sums, one per z plane
  double *mass;
  int nx, ny, nz, pitch;
  int storage;         // 0 FP64, 1 FP32
  int tiles_x, tiles_y;  // 64 x 4 node tiles of one z plane
  int trt;               // two relaxation times (else BGK: tau_m = tau)
  double rho0, tau, omega, gx, gy, gz;
  double tau_m, omega_m;  // relaxation of the antisymmetric parts
  float rho0_f, tau_f, omega_f, gx_f, gy_f, gz_f;
  float tau_m_f, omega_m_f;
};

template <class R> __device__ __forceinline__ R par3(double a, float b);
template <> __device__ __forceinline__ double par3<double>(double a, float) { return a; }
template <> __device__ __forceinline__ float par3<float>(double, float b) { return b; }
__device__ __forceinline__ float fmr(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmr(double a, double b, double c) { return __builtin_fma(a, b, c); }

// BGK or TRT collision of one node in deviation form.  The equilibrium of
// Eq. LB2 with u = J / rho, J = j + rho tau_m g (tau_m = tau for BGK):
// opposite velocities share the even part c and take c +- 3 w (e.J); the
// rest population is delta rho less the other eighteen.  BGK relaxes every
// d_i with omega; TRT relaxes the part of (feq - d) symmetric over a pair
// with omega and the antisymmetric part with omega_m (the rest population is
// symmetric).  FP32 arithmetic forms the increment and gives it exactly the
// method's mass (zero) and momentum (rho g) from sums of the small
// increments before the one final rounding, as the D2Q9 sweep does (the
// momentum term of the stored values would otherwise round the body force
// of slow flows with a bias).
template <class R> __device__ __forceinline__ void collide3(const Dom3 &D, R d[19]) {
  R drho = d[0];
#pragma unroll
  for (int i = 1; i < 19; i += 2) drho += d[i] + d[i + 1];
  R jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 1; i < 19; i += 2) {
    const R o = d[i] - d[i + 1];  // e_{i+1} = -e_i
    if (ex(i)) jx += R(ex(i)) * o;
    if (ey(i)) jy += R(ey(i)) * o;
    if (ez(i)) jz += R(ez(i)) * o;
  }
  const R rho = par3<R>(D.rho0, D.rho0_f) + drho;
  const R irho = R(1) / rho;
  const R tau = par3<R>(D.tau_m, D.tau_m_f), om = par3<R>(D.omega, D.omega_f);
  const R omm = par3<R>(D.omega_m, D.omega_m_f);
  const R gx = par3<R>(D.gx, D.gx_f), gy = par3<R>(D.gy, D.gy_f), gz = par3<R>(D.gz, D.gz_f);
  const R rt = rho * tau;
  const R Jx = fmr(rt, gx, jx), Jy = fmr(rt, gy, jy), Jz = fmr(rt, gz, jz);
  const R ux = Jx * irho, uy = Jy * irho, uz = Jz * irho;
  const R q = (R(1.5) * rho) * fmr(ux, ux, fmr(uy, uy, uz * uz));
  const R r45 = R(4.5) * rho;
  R eq[19];
#pragma unroll
  for (int i = 1; i < 19; i += 2) {
    const R w = i <= 6 ? R(1) / R(18) : R(1) / R(36);
    const R eu = R(ex(i)) * ux + R(ey(i)) * uy + R(ez(i)) * uz;
    const R eJ = R(ex(i)) * Jx + R(ey(i)) * Jy + R(ez(i)) * Jz;
    const R c = w * (drho + fmr(r45 * eu, eu, -q));
    const R l = (R(3) * w) * eJ;
    eq[i] = c + l;
    eq[i + 1] = c - l;
  }
  if constexpr (sizeof(R) == 4) {
    R inc[19];
    if (D.trt) {
#pragma unroll
      for (int i = 1; i < 19; i += 2) {
        const R a = eq[i] - d[i], b = eq[i + 1] - d[i + 1];
        const R sym = R(0.5) * (a + b), anti = R(0.5) * (a - b);
        inc[i] = fmr(om, sym, omm * anti);
        inc[i + 1] = fmr(om, sym, -(omm * anti));
      }
    } else {
#pragma unroll
      for (int i = 1; i < 19; ++i) inc[i] = om * (eq[i] - d[i]);
    }
    R sx = R(0), sy = R(0), sz = R(0);
#pragma unroll
    for (int i = 1; i < 19; i += 2) {
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
    for (int i = 1; i < 19; i += 2) m += inc[i] + inc[i + 1];
    inc[0] = -m;
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = d[i] + inc[i];
  } else {
    R s = R(0);
#pragma unroll
    for (int i = 1; i < 19; i += 2) s += eq[i] + eq[i + 1];
    eq[0] = drho - s;
    if (D.trt) {
      d[0] = fmr(om, eq[0] - d[0], d[0]);
#pragma unroll
      for (int i = 1; i < 19; i += 2) {
        const R a = eq[i] - d[i], b = eq[i + 1] - d[i + 1];
        const R sym = R(0.5) * (a + b), anti = R(0.5) * (a - b);
        d[i] += fmr(om, sym, omm * anti);
        d[i + 1] += fmr(om, sym, -(omm * anti));
      }
    } else {
#pragma unroll
      for (int i = 0; i < 19; ++i) d[i] = fmr(om, eq[i] - d[i], d[i]);
    }
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

// One step of every node: 256 threads = a tile of 64 (x) by 4 (y) nodes of
// one z plane; each wave reads 64 consecutive x of a row per population
// plane.  A solid node stores zero deviations (every slot is written each
// step and never pulled).  Element offsets are 32-bit (the host admits no
// buffer of 2^31 elements or more).
template <int ST>
__global__ __launch_bounds__(256) void k_sweep3(const Dom3 *__restrict__ Dp, int kstep) {
  using T = typename std::conditional<ST == 0, double, float>::type;
  using R = T;
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
  const uint64_t T0 = *D.tstep + (uint64_t)kstep;  // state time of the source buffer
  const T *src = (const T *)D.f[T0 & 1];
  T *dst = (T *)D.f[(T0 + 1) & 1];
  const uint32_t plane = (uint32_t)nz * (uint32_t)ny * (uint32_t)pitch;
  const uint32_t here = ((uint32_t)z * (uint32_t)ny + (uint32_t)y) * (uint32_t)pitch + (uint32_t)x;
  const uint32_t w = D.nodew ? D.nodew[here] : 0u;
  R d[19];
  if (w & NODE_SOLID3) {
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = R(0);
  } else {
    const int xp = x + 1 < nx ? x + 1 : 0, xm = x > 0 ? x - 1 : nx - 1;
    const int yp = y + 1 < ny ? y + 1 : 0, ym = y > 0 ? y - 1 : ny - 1;
    const int zp = z + 1 < nz ? z + 1 : 0, zm = z > 0 ? z - 1 : nz - 1;
    d[0] = src[here];
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      // source x - e_i
      const int sx = ex(i) > 0 ? xm : (ex(i) < 0 ? xp : x);
      const int sy = ey(i) > 0 ? ym : (ey(i) < 0 ? yp : y);
      const int sz = ez(i) > 0 ? zm : (ez(i) < 0 ? zp : z);
      const uint32_t from =
          ((w >> (i - 1)) & 1u)
              ? (uint32_t)opp(i) * plane + here  // halfway bounce-back
              : (uint32_t)i * plane + ((uint32_t)sz * (uint32_t)ny + (uint32_t)sy) * (uint32_t)pitch +
                    (uint32_t)sx;
      d[i] = src[from];
    }
    collide3<R>(D, d);
    if (!(fabs((double)d[0]) < 1e30)) atomicOr(D.health, 1u);
  }
#pragma unroll
  for (int i = 0; i < 19; ++i) dst[(uint32_t)i * plane + here] = d[i];
}

// Node words from the solid mask ([nz][ny][pitch] bytes, 1 = solid).
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
    for (int i = 1; i < 19; ++i)
      if (at(x - ex(i), y - ey(i), z - ez(i))) w |= 1u << (i - 1);
  }
  D.nodew[((size_t)z * D.ny + y) * D.pitch + x] = w;
}

// Equilibrium of the given fields (or rest) as the initial post-collision
// state, after one collision (as the D2Q9 domains start).  Nodes n0 .. n0 +
// cnt - 1; the fields (or null: rest) hold those nodes, [cnt] each.
template <int ST>
__global__ __launch_bounds__(256) void k_init3(const Dom3 *__restrict__ Dp, const double *rho_f,
                                               const double *ux_f, const double *uy_f,
                                               const double *uz_f, long long n0, long long cnt) {
  using T = typename std::conditional<ST == 0, double, float>::type;
  using R = T;
  const Dom3 &D = *Dp;
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= cnt) return;
  const long long n = n0 + k;
  const int x = (int)(n % D.nx), y = (int)((n / D.nx) % D.ny), z = (int)(n / ((long long)D.nx * D.ny));
  const size_t plane = (size_t)D.nz * D.ny * D.pitch;
  const size_t here = ((size_t)z * D.ny + y) * D.pitch + x;
  T *dst = (T *)D.f[*D.tstep & 1];
  const bool solid = D.nodew && (D.nodew[here] & NODE_SOLID3);
  R d[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) d[i] = R(0);
  if (rho_f && !solid) {
    const double r = rho_f[k], vx = ux_f[k], vy = uy_f[k], vz = uz_f[k];
    const double uu = vx * vx + vy * vy + vz * vz;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const double w = i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
      const double eu = ex(i) * vx + ey(i) * vy + ez(i) * vz;
      d[i] = (R)(w * ((r - D.rho0) + r * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu)));
    }
  }
  if (!solid) collide3<R>(D, d);
#pragma unroll
  for (int i = 0; i < 19; ++i) dst[(size_t)i * plane + here] = d[i];
}

// rho and u = j/rho + g/2 of the pre-collision state, recovered from f*:
// collision keeps rho and adds rho g to j.
// Nodes n0 .. n0 + cnt - 1 (x fastest) into out [4][cnt].
template <int ST>
__global__ __launch_bounds__(256) void k_moments3(const Dom3 *__restrict__ Dp, double *out,
                                                  long long n0, long long cnt) {
  using T = typename std::conditional<ST == 0, double, float>::type;
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
  for (int i = 0; i < 19; ++i) {
    const double v = (double)src[(size_t)i * plane + here];
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

// Populations of nodes n0 .. n0 + cnt - 1 as FP64 deviations, out [19][cnt].
template <int ST>
__global__ __launch_bounds__(256) void k_export3(const Dom3 *__restrict__ Dp, double *out,
                                                 long long n0, long long cnt) {
  using T = typename std::conditional<ST == 0, double, float>::type;
  const Dom3 &D = *Dp;
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= cnt) return;
  const long long n = n0 + k;
  const int x = (int)(n % D.nx), y = (int)((n / D.nx) % D.ny), z = (int)(n / ((long long)D.nx * D.ny));
  const size_t plane = (size_t)D.nz * D.ny * D.pitch;
  const size_t here = ((size_t)z * D.ny + y) * D.pitch + x;
  const T *src = (const T *)D.f[*D.tstep & 1];
#pragma unroll
  for (int i = 0; i < 19; ++i) out[(size_t)i * cnt + k] = (double)src[(size_t)i * plane + here];
}

// FP64 density sum: block z sums plane z in a fixed order; one wave adds the
// planes.  Latches a non-finite total.
template <int ST>
__global__ __launch_bounds__(256) void k_mass3_partial(const Dom3 *__restrict__ Dp) {
  using T = typename std::conditional<ST == 0, double, float>::type;
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
      for (int i = 0; i < 19; ++i) r += (double)src[(size_t)i * plane + here];
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
